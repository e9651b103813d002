"""GPU adjoint (vector-Jacobian product) checks.

* J^T w from the HIP reverse kernels against the transpose of the oracle's
  dense complex-step Jacobian on tiny meshes (1e-12 relative);
* the dot-product identity v . (J u) = (J^T v) . u with J u from the oracle's
  complex step, on the 32x32x8 wall / far-field mesh (1e-10 relative);
* torch.autograd through FRResidual: the gradient of a wall pressure force
  after one explicit residual update, L(U) = F_wall(U + tau R(U)), against
  central finite differences on 50 seeded directions; and forward-mode AD
  (FRResidual.jvp) against the exact tangent.
"""
import math

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


def _tiny(kind):
    if kind == "ns_wall_p1to3":
        return I.case_ns_mixed(2, 2, 2, k=51, lengths=(1.0, 1.0, 0.5), wall=True, pvals=(1, 2, 3), pw=(1, 1, 1),
                               re=50.0, ma=0.3)
    if kind == "ns_periodic_p1to4_rusanov":
        c = I.case_ns_mixed(2, 2, 1, k=52, lengths=(1.0, 1.0, 0.5), pvals=(1, 2, 3, 4), pw=(1, 1, 1, 1),
                            re=80.0, ma=0.3)
        c.flux = 1
        return c
    c = I.case_ns_mixed(2, 2, 2, k=53, lengths=(1.0, 1.0, 1.0), pvals=(1, 2, 3), pw=(1, 1, 1), ma=0.3)
    c.physics = 0
    return c


@pytest.mark.parametrize("fused", [False, True], ids=["per_bucket", "fused"])
@pytest.mark.parametrize("kind", ["ns_wall_p1to3", "ns_periodic_p1to4_rusanov", "euler_periodic_p1to3_roe"])
def test_vjp_matches_dense_jacobian(frx, oracle_mod, kind, fused):
    print("case", kind, "fused", fused, flush=True)
    case = _tiny(kind)
    orc = oracle_mod.Oracle.from_case(case)
    ctx = frx.Context.from_case(case)
    ctx.set_launch(fused)
    J = orc.jacobian(case.U)
    U = torch.tensor(case.U, device="cuda")
    for seed in (1, 2):
        w = np.random.default_rng(600 + seed).normal(size=case.U.shape)
        got = ctx.vjp(U, torch.tensor(w, device="cuda")).cpu().numpy()
        ref = (J.T @ w.ravel()).reshape(case.U.shape)
        err = rel_err(got, ref)
        print(kind, "vjp rel err", err)
        assert err <= 1e-12


@pytest.mark.parametrize("fused", [False, True], ids=["per_bucket", "fused"])
def test_dot_product_identity_wall_32x32x8(frx, oracle_mod, fused):
    case = I.config(4)
    orc = oracle_mod.Oracle.from_case(case)
    ctx = frx.Context.from_case(case)
    ctx.set_launch(fused)
    U = torch.tensor(case.U, device="cuda")
    for seed in range(3):
        rng = np.random.default_rng(4400 + seed)
        u = rng.normal(size=case.U.shape)
        v = rng.normal(size=case.U.shape)
        Ju = orc.jvp(case.U, u)
        JTv = ctx.vjp(U, torch.tensor(v, device="cuda")).cpu().numpy()
        lhs = float(np.sum(v * Ju))
        rhs = float(np.sum(JTv * u))
        scale = np.sqrt(np.sum((v * Ju) ** 2)) * math.sqrt(v.size)
        print("dot identity", lhs, rhs, abs(lhs - rhs) / abs(lhs))
        assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), scale * 1e-3)
        # and the GPU's own tangent
        Jg = ctx.jvp(U, torch.tensor(u, device="cuda")).cpu().numpy()
        assert abs(float(np.sum(v * Jg)) - rhs) <= 1e-10 * max(abs(lhs), scale * 1e-3)


def _wall_force_operator(case, oracle_mod):
    """Sparse map from the pressure at solution points to the wall pressure
    force: sum over wall face points of w_a w_b |S| p extrapolated to y = 0."""
    off = I.sp_offsets(case.elem_p)
    rows, cols, vals = [], [], []
    nbr = case.mesh["elem_nbr"]
    xyz = case.mesh["elem_xyz"]
    for e in np.nonzero(nbr[:, 2] == I.BC_WALL)[0]:
        n = int(case.elem_p[e]) + 1
        o = oracle_mod.ops1d(n)
        X = xyz[e]
        hx = np.linalg.norm(X[1] - X[0])
        hz = np.linalg.norm(X[4] - X[0])
        area = 0.25 * hx * hz  # flat, axis-aligned wall face (its vertices are not perturbed)
        for b in range(n):
            for a in range(n):
                for m in range(n):
                    k = a + n * (m + n * b)
                    cols.append(off[e] + k)
                    vals.append(o["w"][a] * o["w"][b] * area * o["lm"][m])
    return np.asarray(cols), np.asarray(vals)


def test_autograd_wall_force_gradient(frx, oracle_mod):
    case = I.config(4)
    ctx = frx.Context.from_case(case)
    cols, vals = _wall_force_operator(case, oracle_mod)
    cols_t = torch.tensor(cols, device="cuda")
    vals_t = torch.tensor(vals, device="cuda")
    tau = 1e-3
    gm1 = case.gamma - 1.0

    def L(U):
        Ut = U + tau * frx.residual(U, ctx)
        p = gm1 * (Ut[4] - 0.5 * (Ut[1] ** 2 + Ut[2] ** 2 + Ut[3] ** 2) / Ut[0])
        return torch.sum(vals_t * p[cols_t])

    U0 = torch.tensor(case.U, device="cuda", requires_grad=True)
    val = L(U0)
    (g,) = torch.autograd.grad(val, U0)
    g = g.detach()
    rng = np.random.default_rng(4444)
    errs = []
    with torch.no_grad():
        Ud = U0.detach()
        for i in range(50):
            d = torch.tensor(rng.normal(size=case.U.shape), device="cuda")
            d /= d.norm()
            # fourth-order central difference at h = 1e-3: truncation O(h^4),
            # and ten times less rounding noise than at h = 1e-4 (where the
            # rounding of L, divided by h, is about 1e-7 of the product)
            h = 1e-3
            fd = (8.0 * (L(Ud + h * d) - L(Ud - h * d)).item() - (L(Ud + 2 * h * d) - L(Ud - 2 * h * d)).item()) / (12 * h)
            ad = torch.sum(g * d).item()
            errs.append(abs(fd - ad) / max(abs(ad), 1e-30))
    errs = np.array(errs)
    print("autograd vs fourth-order central FD: median", np.median(errs), "max", errs.max())
    assert np.median(errs) <= 1e-7 and errs.max() <= 1e-5


def test_forward_mode_matches_exact_tangent(frx, oracle_mod):
    import torch.autograd.forward_ad as fwAD
    case = _tiny("ns_wall_p1to3")
    ctx = frx.Context.from_case(case)
    orc = oracle_mod.Oracle.from_case(case)
    U = torch.tensor(case.U, device="cuda")
    v = np.random.default_rng(9).normal(size=case.U.shape)
    with fwAD.dual_level():
        Ud = fwAD.make_dual(U, torch.tensor(v, device="cuda"))
        R = frx.residual(Ud, ctx)
        t = fwAD.unpack_dual(R).tangent
    assert rel_err(t.cpu().numpy(), orc.jvp(case.U, v)) <= 1e-12
