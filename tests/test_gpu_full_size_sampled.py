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
extended-precision evaluation); exact float64 tangent within 1e-12; float32
tangent within 1e-3 of the exact one (float32 storage and accumulation).
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


@pytest.fixture(scope="module", params=["box_128x128x8_re60000", "street_64x64x8_indicator"])
def full(request, frx):
    name = request.param
    print("full-size case", name, flush=True)
    if name.startswith("box"):
        case = I.config(5)
    else:
        from paper_1910_03693_amd import adapt
        p, hist = adapt.indicator_degree_field(lambda ep: I.case_street(elem_p=ep))
        print("degree histogram per sweep", hist, flush=True)
        case = I.case_street(elem_p=p)
    ctx = frx.Context.from_case(case)
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
    Ro, Rl, Jo, Rg, Jg, J32g = [], [], [], [], [], []
    for e in els:
        sub, cols = patch_case(case, e, off)
        po = oracle_mod.Oracle.from_case(sub)
        n3 = int(off[e + 1] - off[e])
        blk = element_block(case, e, off)
        Ro.append(po.residual(sub.U)[:, :n3])
        Rl.append(po.residual_ld(sub.U)[:, :n3])
        Jo.append(po.jvp(sub.U, v[:, cols])[:, :n3])
        Rg.append(R[:, blk])
        Jg.append(Jv[:, blk])
        J32g.append(J32[:, blk])
    cat = lambda xs: np.concatenate(xs, axis=1)
    Ro, Rl, Jo, Rg, Jg, J32g = map(cat, (Ro, Rl, Jo, Rg, Jg, J32g))
    floor = rel_err(Ro, Rl)
    err, err_ld = rel_err(Rg, Ro), rel_err(Rg, Rl)
    ej, e32 = rel_err(Jg, Jo), rel_err(J32g, Jo)
    print(f"{name}: {len(els)} elements (degrees {sorted(set(case.elem_p[els].tolist()))}); residual rel err "
          f"{err:.3e} (vs extended {err_ld:.3e}, oracle floor {floor:.3e}); exact tangent {ej:.3e}; "
          f"float32 tangent {e32:.3e}")
    tol = max(1e-12, 4 * floor)
    assert err <= tol and err_ld <= tol
    assert ej <= 1e-12
    assert e32 <= 1e-3
