"""Nodal polynomial filter on the GPU (section 4.2) against the oracle's
filter: mixed degrees 1..5 with ragged buckets, in place and out of place,
the paper's setting (p > 2, alpha = 0.2) and the edge cases (alpha 0 and 1,
every degree filtered, no element filtered, invalid arguments)."""
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


@pytest.fixture(scope="module")
def case():
    m = I.box_mesh(7, 5, 3, (1.4, 1.0, 0.6), noise=0.03, seed=81)
    p = I.draw_p(m["n_elem"], [1, 2, 3, 4, 5], [1, 1, 1, 1, 1], 82)
    modes = I.FourierModes((1.4, 1.0, 0.6), 2 * np.pi * 4, 0.2, 83)
    U = I.sample(m, p, lambda x, y, z: I.perturbed_uniform_flow(x, y, z, modes, 0.3))
    return I.Case("t", m, p, U, 1, 0, 1.4, 1e-2, 0.72, I._farfield(0.3), {})


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("alpha,p_from", [(0.2, 3), (0.5, 1), (1.0, 2), (0.2, 5)])
@pytest.mark.parametrize("in_place", [False, True], ids=["out", "in_place"])
def test_filter_matches_oracle(frx, case, alpha, p_from, in_place):
    from oracle import filter as OF
    print("alpha", alpha, "p_from", p_from, "in_place", in_place, flush=True)
    ctx = frx.Context.from_case(case)
    U = torch.tensor(case.U, device="cuda")
    if in_place:
        got = U.clone()
        ctx.nodal_filter(got, alpha, p_from, out=got)
    else:
        got = ctx.nodal_filter(U, alpha, p_from)
    got = got.cpu().numpy()
    ref = OF.nodal_filter(case.elem_p, case.U, alpha, p_from)
    err = _rel(got, ref)
    print("rel err", err)
    assert err <= 1e-13
    # elements below p_from are copied bit for bit
    n = case.elem_p.astype(np.int64) + 1
    off = np.concatenate([[0], np.cumsum(n ** 3)])
    for e in np.nonzero(case.elem_p < p_from)[0]:
        np.testing.assert_array_equal(got[:, off[e]:off[e + 1]], case.U[:, off[e]:off[e + 1]])
    # the input is left alone out of place
    if not in_place:
        np.testing.assert_array_equal(U.cpu().numpy(), case.U)


def test_alpha_zero_is_the_identity(frx, case):
    ctx = frx.Context.from_case(case)
    U = torch.tensor(case.U, device="cuda")
    np.testing.assert_array_equal(ctx.nodal_filter(U, 0.0, 1).cpu().numpy(), case.U)


def test_invalid_arguments(frx, case):
    ctx = frx.Context.from_case(case)
    U = torch.tensor(case.U, device="cuda")
    for alpha, p_from in [(-0.1, 3), (1.5, 3), (float("nan"), 3), (0.2, 0), (0.2, 6)]:
        with pytest.raises(frx.FrError) as ei:
            ctx.nodal_filter(U, alpha, p_from)
        assert ei.value.status == -1
    # an output that overlaps the input without being it is refused
    big = torch.zeros(2 * U.numel(), dtype=torch.float64, device="cuda")
    big[:U.numel()] = U.reshape(-1)
    src = big[:U.numel()].view_as(U)
    dst = big[7:7 + U.numel()].view_as(U)
    with pytest.raises(frx.FrError) as ei:
        ctx.nodal_filter(src, 0.2, 3, out=dst)
    assert ei.value.status == -1


def test_full_size_workload(frx):
    """The 32x32x4 Navier-Stokes workload (4096 elements, p 1..4), the
    paper's setting."""
    from oracle import filter as OF
    c2 = I.config(2)
    ctx = frx.Context.from_case(c2)
    U = torch.tensor(c2.U, device="cuda")
    got = ctx.nodal_filter(U, 0.2, 3).cpu().numpy()
    ref = OF.nodal_filter(c2.elem_p, c2.U, 0.2, 3)
    err = _rel(got, ref)
    print("32x32x4 rel err", err)
    assert err <= 1e-13
