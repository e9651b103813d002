"""Parity at full size on sampled elements.

The 128x128x8 Re 60000 box (29.6 M DOF) and the 64x64x8 vortex street with
its indicator-chosen degree field (12.7 M DOF) are too large for the oracle to
evaluate whole in a test.  The GPU computes R(U), the exact float64 tangent
and the float32 tangent on the full mesh, in the fused launch the benchmark
times; the oracle evaluates the same quantities on the patch of each sampled
element (the element and its face neighbours, which fix its residual block;
the patch construction is pinned on the CPU in test_patches.py).

Tolerances as for the whole-mesh tests: float64 residual within
max(1e-12, 4 x the oracle's own float64 rounding floor against its
extended-precision evaluation), and its error relative to the largest sum of
absolute terms (the scale at which its rounding happens) reported and bounded
by 1e-13; exact float64 tangent within 1e-12; float32 tangent within 1e-4 of
the exact one (float32 storage and accumulation).

The vortex street's degree field, chosen on the device, is also compared in
full with the one the oracle's indicator, criteria and limiter choose on the
whole 64x64x8 mesh (integer result: bit-exact).  And on the 128x128x8 box one
implicit ESDIRK2 stage (GMRES(30) to 1e-6, PTC to 1e-4) in the mixed form
(float32 exact tangent and basis) is compared with the same stage in float64:
the oracle cannot solve this stage in a test's time, so the reference is the
float64 GPU path, whose operators are the ones checked against the oracle
above.  The same holds for one full ESDIRK2 step of the vortex street on its
indicator degree field (measured: 1.2e-8 relative, against a change of U by
4.4e-3 over the step).
"""
import numpy as np
import pytest

from paper_1910_03693_amd import inputs as I

from patches import element_block, patch_case, sample_elements

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel_err(a, b):
    a = np.asarray(a).reshape(5, -1)
    b = np.asarray(b).reshape(5, -1)
    big = np.abs(b).max()
    out = np.abs(a - b).max() / big
    for v in range(5):
        s = np.abs(b[v]).max()
        if s >= 1e-3 * big:
            out = max(out, np.abs(a[v] - b[v]).max() / s)
    return out


@pytest.fixture(scope="module")
def frx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_03693_amd import frx as F
    F.lib()
    return F


@pytest.fixture(scope="module")
def street_degrees(frx):
    from paper_1910_03693_amd import adapt
    p, hist = adapt.indicator_degree_field(lambda ep: I.case_street(elem_p=ep))
    print("degree histogram per sweep", hist, flush=True)
    return p, hist


@pytest.fixture(scope="module", params=["box_128x128x8_re60000", "street_64x64x8_indicator"])
def full(request, frx, street_degrees):
    name = request.param
    print("full-size case", name, flush=True)
    if name.startswith("box"):
        case = I.config(5)
    else:
        case = I.case_street(elem_p=street_degrees[0])
    ctx = frx.Context.from_case(case, max_restart=0)
    ctx.set_launch(True)
    U = torch.tensor(case.U, device="cuda")
    v = I.random_direction(case.U.size, 4005).reshape(case.U.shape)
    vt = torch.tensor(v, device="cuda")
    print(name, "dof", ctx.n_dof, "residual and tangents on the GPU", flush=True)
    R = ctx.residual(U).cpu().numpy()
    Jv = ctx.jvp(U, vt).cpu().numpy()
    J32 = ctx.jvp(U, vt.float(), precision=frx.FR_F32).double().cpu().numpy()
    assert ctx.nonphysical() == 0
    ctx.close()
    del U, vt
    torch.cuda.empty_cache()
    return name, case, v, R, Jv, J32


def test_sampled_blocks_match_oracle_patches(full, oracle_mod):
    name, case, v, R, Jv, J32 = full
    off = I.sp_offsets(case.elem_p)
    els = sample_elements(case.elem_p, 6, 707)
    Ro, Rl, Jo, Rg, Jg, J32g, To = [], [], [], [], [], [], []
    for e in els:
        sub, cols = patch_case(case, e, off)
        po = oracle_mod.Oracle.from_case(sub)
        n3 = int(off[e + 1] - off[e])
        blk = element_block(case, e, off)
        r_o, t_o = po.residual_terms(sub.U)
        Ro.append(r_o[:, :n3])
        To.append(t_o[:, :n3])
        Rl.append(po.residual_ld(sub.U)[:, :n3])
        Jo.append(po.jvp(sub.U, v[:, cols])[:, :n3])
        Rg.append(R[:, blk])
        Jg.append(Jv[:, blk])
        J32g.append(J32[:, blk])
    cat = lambda xs: np.concatenate(xs, axis=1)
    Ro, Rl, Jo, Rg, Jg, J32g, To = map(cat, (Ro, Rl, Jo, Rg, Jg, J32g, To))
    floor = rel_err(Ro, Rl)
    err, err_ld = rel_err(Rg, Ro), rel_err(Rg, Rl)
    # error relative to the largest sum of absolute terms, per variable
    err_terms = max(np.abs(Rg[v] - Rl[v]).max() / To[v].max() for v in range(5))
    ej, e32 = rel_err(Jg, Jo), rel_err(J32g, Jo)
    print(f"{name}: {len(els)} elements (degrees {sorted(set(case.elem_p[els].tolist()))}); residual rel err "
          f"{err:.3e} (vs extended {err_ld:.3e}, oracle floor {floor:.3e}; relative to the summed terms "
          f"{err_terms:.3e}); exact tangent {ej:.3e}; float32 tangent {e32:.3e}")
    tol = max(1e-12, 4 * floor)
    assert err <= tol and err_ld <= tol
    assert err_terms <= 1e-13
    assert ej <= 1e-12
    assert e32 <= 1e-4


def test_street_degree_field_matches_oracle_full_mesh(street_degrees, oracle_mod):
    from oracle import degrees
    p_gpu, hist = street_degrees
    p, hist_o = degrees.indicator_degree_field(
        lambda ep: I.case_street(elem_p=ep), lambda case: oracle_mod.Oracle.from_case(case).indicator(case.U, var=1))
    print("64x64x8 degree histogram (device / oracle):", np.bincount(p_gpu, minlength=6)[1:].tolist(),
          np.bincount(p, minlength=6)[1:].tolist(), hist, hist_o)
    assert np.array_equal(p_gpu.astype(np.int64), p)
    assert hist == hist_o


def test_box_128x128x8_mixed_stage_against_float64_stage(frx):
    case = I.config(5)
    ctx = frx.Context.from_case(case, max_restart=30, graphs=frx.FR_GRAPHS_F64_EXACT | frx.FR_GRAPHS_F32_EXACT)
    ctx.set_launch(True)
    U = torch.tensor(case.U, device="cuda")
    kw = dict(dtau_init=2e-4, dtau_max=4e-3, tol_pseudo=1e-4, max_ptc_iter=60, last_stage=2)
    out = {}
    for name, prec in (("float64", frx.FR_F64), ("mixed", frx.FR_F32)):
        Us = U.clone()
        st = ctx.esdirk_step(Us, 0.002, gmres=dict(restart=30, max_iter=300, tol=1e-6, precision=prec,
                                                  use_graph=True), **kw)
        print("128x128x8 stage", name, st, flush=True)
        assert st["status"] == frx.FR_OK
        out[name] = (Us, st)
    d = (torch.linalg.norm(out["mixed"][0] - out["float64"][0]) / torch.linalg.norm(out["float64"][0])).item()
    change = (torch.linalg.norm(out["float64"][0] - U) / torch.linalg.norm(U)).item()
    print(f"mixed vs float64 stage solution: {d:.3e} relative (the stage changes U by {change:.3e})")
    # both solutions satisfy the same stage equation to the PTC tolerance;
    # they agree far below the change the stage makes
    assert d <= 1e-6 and d <= 1e-3 * change


def test_street_64x64x8_full_step_mixed_against_float64(frx, street_degrees):
    """One full ESDIRK2 step (all three stages) of the vortex street on its
    indicator degree field at the paper's settings (dt 0.05, dtau from dt/10
    up to dt, PTC to 1e-4, GMRES(30) to 1e-1): the mixed form (float32 exact
    tangent and basis, captured graphs) against the float64 exact form.  As
    for the 128x128x8 stage, the reference is the float64 GPU path, whose
    operators are checked against the oracle above; both forms take the same
    pseudo-time path, so they agree to well below the GMRES tolerance's effect
    on the step."""
    case = I.case_street(elem_p=street_degrees[0])
    ctx = frx.Context.from_case(case, max_restart=30, graphs=frx.FR_GRAPHS_F64_EXACT | frx.FR_GRAPHS_F32_EXACT)
    ctx.set_launch(True)
    U = torch.tensor(case.U, device="cuda")
    dt = 0.05
    kw = dict(dtau_init=dt / 10, dtau_max=dt, tol_pseudo=1e-4, max_ptc_iter=60)
    out = {}
    for name, prec in (("float64", frx.FR_F64), ("mixed", frx.FR_F32)):
        Us = U.clone()
        st = ctx.esdirk_step(Us, dt, gmres=dict(restart=30, max_iter=100, tol=1e-1, precision=prec, use_graph=True),
                             **kw)
        print("64x64x8 street step", name, st, flush=True)
        assert st["status"] == frx.FR_OK and st["stages"] == 2
        out[name] = (Us, st)
    d = (torch.linalg.norm(out["mixed"][0] - out["float64"][0]) / torch.linalg.norm(out["float64"][0])).item()
    change = (torch.linalg.norm(out["float64"][0] - U) / torch.linalg.norm(U)).item()
    print(f"mixed vs float64 step: {d:.3e} relative (the step changes U by {change:.3e})")
    assert out["mixed"][1]["ptc_iterations"] == out["float64"][1]["ptc_iterations"]
    assert d <= 1e-6 and d <= 1e-3 * change
    ctx.close()
