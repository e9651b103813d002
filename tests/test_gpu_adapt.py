"""p-adaptation on the GPU (section 3.1): degree selection (indicator,
criteria, face limiter) against the oracle's indicator and the oracle's
criteria and limiter (oracle/degrees.py; integer result: bit-exact), and the
projection of the state between degree fields against the oracle's
projection."""
import numpy as np
import pytest

from paper_1910_03693_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def frx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_03693_amd import frx as F
    F.lib()
    return F


def oracle_degrees(oracle_mod, case, nu_max=0.1, nu_min=0.001, p_min=1, p_max=5, eta_max_scope=0):
    from oracle import degrees
    eta, mx = oracle_mod.Oracle.from_case(case).indicator(case.U, var=1)
    return degrees.select_degrees(case.elem_p, eta, mx, case.mesh["elem_nbr"], nu_max, nu_min, p_min, p_max,
                                  "degree" if eta_max_scope else "all")


def _mixed_case():
    m = I.box_mesh(6, 5, 3, (1.2, 1.0, 0.6), noise=0.02, seed=71)
    p = I.draw_p(m["n_elem"], [1, 2, 3, 4, 5], [1, 1, 1, 1, 1], 72)
    modes = I.FourierModes((1.2, 1.0, 0.6), 2 * np.pi * 3, 0.1, 73)
    U = I.sample(m, p, lambda x, y, z: I.perturbed_uniform_flow(x, y, z, modes, 0.3))
    return I.Case("t", m, p, U, 1, 0, 1.4, 1e-2, 0.72, I._farfield(0.3), {})


@pytest.mark.parametrize("kind,kw", [
    ("street_16x16x2_from_p5", dict()),
    ("street_16x16x2_from_p5_nu", dict(nu_max=0.05, nu_min=0.01, p_min=2, p_max=4)),
    ("mixed_random_p", dict()),
    ("mixed_random_p_p1p2", dict(p_min=1, p_max=2)),
    ("mixed_random_p_same_degree_max", dict(eta_max_scope=1)),
    ("street_16x16x2_mixed_same_degree_max", dict(eta_max_scope=1)),
])
def test_select_degrees_matches_oracle(frx, oracle_mod, kind, kw):
    print("case", kind, kw, flush=True)
    if kind == "street_16x16x2_mixed_same_degree_max":
        case = I.case_street(16, 16, 2, elem_p=I.draw_p(16 * 16 * 2, [1, 2, 3, 4, 5], [1, 1, 1, 1, 1], 77))
    elif kind.startswith("street"):
        case = I.case_street(16, 16, 2, elem_p=np.full(16 * 16 * 2, 5, np.int8))
    else:
        case = _mixed_case()
    ctx = frx.Context.from_case(case)
    U = torch.tensor(case.U, device="cuda")
    args = dict(nu_max=0.1, nu_min=0.001, p_min=1, p_max=5)
    args.update(kw)
    got = ctx.select_degrees(U, 1, **args).cpu().numpy().astype(np.int64)
    ref = oracle_degrees(oracle_mod, case, **args)
    print(kind, "histogram", np.bincount(got, minlength=6)[1:], "changed", int((got != case.elem_p).sum()))
    assert np.array_equal(got, ref)
    nbr = case.mesh["elem_nbr"]
    assert np.all(np.abs(got[:, None] - np.where(nbr >= 0, got[np.clip(nbr, 0, None)], got[:, None])) <= 1)


def test_select_degrees_rejects_bad_arguments(frx):
    case = _mixed_case()
    ctx = frx.Context.from_case(case)
    U = torch.tensor(case.U, device="cuda")
    for kw in (dict(p_min=0), dict(p_max=6), dict(p_min=3, p_max=2), dict(nu_max=1e-4, nu_min=1e-3), dict(var=5)):
        args = dict(var=1, nu_max=0.1, nu_min=0.001, p_min=1, p_max=5)
        args.update(kw)
        with pytest.raises(frx.FrError):
            ctx.select_degrees(U, **args)


def test_projection_matches_oracle(frx, oracle_mod):
    from oracle import projection as P
    case = _mixed_case()
    rng = np.random.default_rng(74)
    for trial in range(3):
        p_new = rng.integers(1, 6, case.mesh["n_elem"]).astype(np.int8)
        print("projection trial", trial, flush=True)
        src = frx.Context.from_case(case)
        dst_case = I.Case("t", case.mesh, p_new, None, case.physics, case.flux, case.gamma, case.mu, case.prandtl,
                          case.farfield, {})
        dst = frx.Context.from_case(dst_case)
        got = src.project_to(torch.tensor(case.U, device="cuda"), dst).cpu().numpy()
        ref = P.project(case.elem_p, case.U, p_new)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print("projection rel err", err)
        assert err <= 1e-13


def test_adapt_step_street(frx, oracle_mod):
    """One adaptation of the vortex street (16x16x2) from p = 5 everywhere:
    degrees as the oracle picks them, state as the oracle projects it."""
    from oracle import projection as P
    from paper_1910_03693_amd import adapt
    case = I.case_street(16, 16, 2, elem_p=np.full(16 * 16 * 2, 5, np.int8))
    ctx = frx.Context.from_case(case)
    U = torch.tensor(case.U, device="cuda")
    new_case, new_ctx, U2 = adapt.adapt_step(case, ctx, U)
    p_ref = oracle_degrees(oracle_mod, case, eta_max_scope=1)  # adapt_step's default reading
    assert np.array_equal(new_case.elem_p.astype(np.int64), p_ref)
    ref = P.project(case.elem_p, case.U, new_case.elem_p)
    assert np.abs(U2.cpu().numpy() - ref).max() <= 1e-13 * np.abs(ref).max()
    # the new context runs: its residual is finite and the state physical
    R = new_ctx.residual(U2)
    assert torch.isfinite(R).all().item() and new_ctx.nonphysical() == 0
