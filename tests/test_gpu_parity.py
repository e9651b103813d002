"""GPU parity: the HIP library (through the C ABI) against the CPU oracle on the
same seeded inputs.

Floating-point tolerances: FP64 residual, exact tangent and indicator within
1e-12 of the oracle's infinity norm per variable; FP32 tangent within 1e-4;
GMRES with a fixed number of iterations within 1e-9; converged solves within
their tolerances.
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
    """max over variables of |a_v - b_v|_inf / |b_v|_inf, skipping variables whose
    reference is below 1e-3 of the largest (they are compared globally)."""
    a = np.asarray(a).reshape(5, -1)
    b = np.asarray(b).reshape(5, -1)
    big = np.abs(b).max()
    out = np.abs(a - b).max() / big
    for v in range(5):
        s = np.abs(b[v]).max()
        if s >= 1e-3 * big:
            out = max(out, np.abs(a[v] - b[v]).max() / s)
    return out


def _tiny_cases():
    cs = {}
    cs["vortex_p2_rusanov"] = I.config(1)
    # The vortex is z-invariant, so at every z-face both sides of Rusanov's
    # max(|u.n| + c) agree up to rounding: a tie where the tangent is not
    # unique.  A small seeded 3-D perturbation removes the ties.
    v = I.config(1)
    pert = I.FourierModes((10.0, 10.0, 2.5), 2 * math.pi * 0.8, 1e-3, 45)
    X = I.solution_points(v.mesh, v.elem_p)
    up = pert(X[0], X[1], X[2])
    U3 = v.U.copy()
    U3[1:4] += U3[0] * up
    cs["vortex_p2_rusanov_3d"] = I.Case("t", v.mesh, v.elem_p, U3, 0, 1, 1.4, 0.0, 0.72, v.farfield, {})
    m = I.box_mesh(3, 3, 2, (1.0, 1.0, 0.6), noise=0.02, seed=41)
    p = I.draw_p(m["n_elem"], [1, 2, 3, 4, 5], [1, 1, 1, 1, 1], 42)
    modes = I.FourierModes((1.0, 1.0, 0.6), 2 * math.pi * 3, 0.1, 43)
    U = I.sample(m, p, lambda x, y, z: I.perturbed_uniform_flow(x, y, z, modes, 0.3))
    cs["mixed_p1to5_ns_roe"] = I.Case("t", m, p, U, 1, 0, 1.4, 1e-2, 0.72, I._farfield(0.3), {})
    cs["mixed_p1to5_ns_rusanov"] = I.Case("t", m, p, U, 1, 1, 1.4, 1e-2, 0.72, I._farfield(0.3), {})
    cs["mixed_p1to5_euler_roe"] = I.Case("t", m, p, U, 0, 0, 1.4, 0.0, 0.72, I._farfield(0.3), {})
    cw = I.case_ns_mixed(3, 4, 2, k=44, lengths=(1.0, 1.0, 0.5), wall=True, re=100.0, ma=0.3)
    cs["wall_farfield_ns_roe"] = cw
    # uniform degree at both ends of the range: p = 1 only (largest tiles),
    # p = 5 only with wall and far field (float64-dual traces one variable at
    # a time)
    mu1 = I.box_mesh(5, 4, 3, (1.0, 0.8, 0.6), noise=0.03, seed=46)
    pu1 = np.ones(mu1["n_elem"], np.int8)
    Uu1 = I.sample(mu1, pu1, lambda x, y, z: I.perturbed_uniform_flow(x, y, z, modes, 0.3))
    cs["uniform_p1_ns_roe"] = I.Case("t", mu1, pu1, Uu1, 1, 0, 1.4, 1e-2, 0.72, I._farfield(0.3), {})
    cu5 = I.case_ns_mixed(2, 2, 2, k=47, lengths=(1.0, 1.0, 0.5), wall=True, pvals=(5,), pw=(1,), re=100.0, ma=0.3)
    cu5.flux = 1
    cs["uniform_p5_ns_rusanov_wall"] = cu5
    m1 = I.box_mesh(1, 1, 1, (1.0, 1.0, 1.0), noise=0.0)
    p1 = np.array([3], np.int8)
    U1 = I.sample(m1, p1, lambda x, y, z: I.perturbed_uniform_flow(x, y, z, modes, 0.3))
    cs["single_self_periodic_ns"] = I.Case("t", m1, p1, U1, 1, 0, 1.4, 1e-2, 0.72, I._farfield(0.3), {})
    return cs


CASES = _tiny_cases()


def _pair(frx, oracle_mod, case, **reserve):
    orc = oracle_mod.Oracle.from_case(case)
    ctx = frx.Context.from_case(case, **reserve)
    U = torch.tensor(case.U, device="cuda")
    return orc, ctx, U


# launch variants: (fused, two-pass Navier-Stokes face stage)
LAUNCH = {"per_bucket": (False, False), "fused": (True, False), "per_bucket_2pass": (False, True),
          "fused_2pass": (True, True)}


@pytest.mark.parametrize("launch", list(LAUNCH))
@pytest.mark.parametrize("name", sorted(CASES))
def test_residual_parity_small(frx, oracle_mod, name, launch):
    print("case", name, "launch", launch, flush=True)
    case = CASES[name]
    orc, ctx, U = _pair(frx, oracle_mod, case)
    ctx.set_launch(*LAUNCH[launch])
    R = ctx.residual(U)
    torch.cuda.synchronize()
    _full_size_residual_check(R.cpu().numpy(), orc, case, name)
    assert ctx.nonphysical() == 0


@pytest.mark.parametrize("launch", list(LAUNCH))
@pytest.mark.parametrize("name", sorted(set(CASES) - {"vortex_p2_rusanov"}))
def test_exact_jvp_parity_small(frx, oracle_mod, name, launch):
    print("case", name, "launch", launch, flush=True)
    case = CASES[name]
    orc, ctx, U = _pair(frx, oracle_mod, case)
    ctx.set_launch(*LAUNCH[launch])
    v = I.random_direction(case.U.size, 4000 + len(name)).reshape(case.U.shape)
    Jv = ctx.jvp(U, torch.tensor(v, device="cuda"))
    torch.cuda.synchronize()
    ref = orc.jvp(case.U, v)
    err = rel_err(Jv.cpu().numpy(), ref)
    print(name, "jvp rel err", err)
    assert err <= 1e-12
    # float32 tangent from a float32 copy of U
    J32 = ctx.jvp(U, torch.tensor(v, device="cuda", dtype=torch.float32), precision=frx.FR_F32)
    e32 = rel_err(J32.double().cpu().numpy(), ref)
    print(name, "fp32 jvp rel err", e32)
    assert e32 <= 1e-4


@pytest.mark.parametrize("fused", [False, True], ids=["per_bucket", "fused"])
@pytest.mark.parametrize("name", ["mixed_p1to5_ns_roe", "wall_farfield_ns_roe", "mixed_p1to5_euler_roe"])
def test_residual_and_tangent_in_one_pass(frx, oracle_mod, name, fused):
    """fr_residual_jvp: the value part of the dual-number pass is the float64
    residual (to the oracle's tolerance, and to the separate residual call),
    its derivative part the exact tangent."""
    print("case", name, "fused", fused, flush=True)
    case = CASES[name]
    orc, ctx, U = _pair(frx, oracle_mod, case)
    ctx.set_launch(fused)
    v = I.random_direction(case.U.size, 4100 + len(name)).reshape(case.U.shape)
    R, Jv = ctx.residual_jvp(U, torch.tensor(v, device="cuda"))
    torch.cuda.synchronize()
    _full_size_residual_check(R.cpu().numpy(), orc, case, name + " residual (one pass)")
    assert rel_err(Jv.cpu().numpy(), orc.jvp(case.U, v)) <= 1e-12
    R1 = ctx.residual(U).cpu().numpy()
    assert rel_err(R.cpu().numpy(), R1) <= 1e-13


@pytest.fixture(scope="module")
def c2(frx, oracle_mod):
    case = I.config(2)
    orc, ctx, U = _pair(frx, oracle_mod, case)
    return case, orc, ctx, U


def _full_size_residual_check(R, orc, case, label):
    """1e-12 relative to the oracle, unless the oracle's own float64 rounding
    error (against its extended-precision evaluation of the same
    discretisation) is larger: at Mach 0.1-0.2 the momentum residual is a small
    difference of terms of size p_inf (p+1)^2 / h.  Then the GPU must sit
    within 4x of that rounding floor, from the oracle and from the
    extended-precision value."""
    Ro = orc.residual(case.U)
    Rl = orc.residual_ld(case.U)
    floor = rel_err(Ro, Rl)
    err = rel_err(R, Ro)
    err_ld = rel_err(R, Rl)
    glob = np.abs(R - Ro).max() / np.abs(Ro).max()
    print(f"{label}: rel err vs oracle {err:.3e} (global {glob:.3e}), vs extended precision {err_ld:.3e}, "
          f"oracle rounding floor {floor:.3e}")
    tol = max(1e-12, 4 * floor)
    assert err <= tol
    assert err_ld <= tol


@pytest.mark.parametrize("launch", list(LAUNCH))
def test_residual_parity_ns_mixed_32x32x4(frx, c2, launch):
    case, orc, ctx, U = c2
    ctx.set_launch(*LAUNCH[launch])
    R = ctx.residual(U)
    torch.cuda.synchronize()
    _full_size_residual_check(R.cpu().numpy(), orc, case, "c2 residual")


def test_residual_and_tangent_in_one_pass_32x32x4(frx, c2):
    case, orc, ctx, U = c2
    ctx.set_launch(True)
    v = I.random_direction(case.U.size, 4002).reshape(case.U.shape)
    R, Jv = ctx.residual_jvp(U, torch.tensor(v, device="cuda"))
    torch.cuda.synchronize()
    _full_size_residual_check(R.cpu().numpy(), orc, case, "c2 residual (one pass)")
    err = rel_err(Jv.cpu().numpy(), orc.jvp(case.U, v))
    print("c2 one-pass tangent rel err", err)
    assert err <= 1e-12


@pytest.mark.parametrize("launch", list(LAUNCH))
def test_jvp_parity_ns_mixed_32x32x4(frx, c2, launch):
    case, orc, ctx, U = c2
    ctx.set_launch(*LAUNCH[launch])
    v = I.random_direction(case.U.size, 4002).reshape(case.U.shape)
    vt = torch.tensor(v, device="cuda")
    ref = orc.jvp(case.U, v)
    Jv = ctx.jvp(U, vt)
    e64 = rel_err(Jv.cpu().numpy(), ref)
    J32 = ctx.jvp(U, vt.float(), precision=frx.FR_F32)
    e32 = rel_err(J32.double().cpu().numpy(), ref)
    Jfd = ctx.jvp(U, vt, jv_mode=frx.FR_JV_FD, fd_eps=1e-6)
    efd = rel_err(Jfd.cpu().numpy(), ref)
    ofd = orc.jvp_fd(case.U, v, 1e-6)
    print("c2 jvp rel err: exact fp64", e64, "fp32", e32, "fd", efd, "oracle fd", rel_err(ofd, ref))
    assert e64 <= 1e-12
    assert e32 <= 1e-4
    # finite differences carry O(eps) truncation and O(u/eps) rounding: both
    # implementations sit at the same distance from the exact product
    assert efd <= 1e-5 and abs(efd - rel_err(ofd, ref)) <= 1e-5


def _fd_floor(orc, U, vu, eps):
    """Rounding noise of a float64 finite difference on these inputs: the
    oracle's float64 difference against the same difference of its
    extended-precision residuals (same perturbed state)."""
    Up = U + eps * vu
    fd_ld = (orc.residual_ld(Up) - orc.residual_ld(U)) / eps
    return rel_err(orc.jvp_fd(U, vu, eps), fd_ld)


@pytest.mark.parametrize("mode", ["fd", "fd_scaled"])
@pytest.mark.parametrize("name", ["vortex_1", "ns_mixed_32x32x4"])
def test_fd_jvp_matches_oracle_fd_elementwise(frx, oracle_mod, name, mode):
    """fr_jvp(FR_JV_FD / FR_JV_FD_SCALED) against the oracle's finite
    difference at the same step along the unit direction (eps = 1e-6, or
    1e-6 sqrt(1 + ||U||) scaled), element by element.  Both sides round R to
    float64 and the difference divides that rounding by the step, so the bound
    is max(1e-7, 4x the oracle's own rounding noise of the difference)."""
    case = CASES["vortex_p2_rusanov_3d"] if name == "vortex_1" else I.config(2)
    print("case", name, mode, flush=True)
    orc, ctx, U = _pair(frx, oracle_mod, case, max_restart=0)
    ctx.set_launch(True)
    v = I.random_direction(case.U.size, 4010).reshape(case.U.shape)
    nv = np.linalg.norm(v)
    eps = 1e-6 if mode == "fd" else 1e-6 * math.sqrt(1.0 + np.linalg.norm(case.U))
    jv = frx.FR_JV_FD if mode == "fd" else frx.FR_JV_FD_SCALED
    got = ctx.jvp(U, torch.tensor(v, device="cuda"), jv_mode=jv, fd_eps=1e-6).cpu().numpy()
    ref = orc.jvp_fd(case.U, v / nv, eps) * nv
    floor = _fd_floor(orc, case.U, v / nv, eps)
    err = rel_err(got, ref)
    exact = rel_err(got, orc.jvp(case.U, v))
    print(f"{name} {mode}: rel err vs oracle fd {err:.3e} (rounding floor {floor:.3e}); vs exact {exact:.3e}")
    assert err <= max(1e-7, 4 * floor)


def test_esdirk_forced_halving_matches_oracle(frx, oracle_mod):
    """A GMRES budget too small for the first pseudo time step: both sides
    halve dtau the same number of times in each iterate and reach the same
    stage solution."""
    case = CASES["vortex_p2_rusanov"]
    orc, ctx, U = _pair(frx, oracle_mod, case)
    kw = dict(dtau_init=2.0, dtau_max=2.0, dtau_min=2.0 / 2 ** 12, tol_pseudo=1e-8, last_stage=2)
    Uo, so = orc.esdirk2_step(case.U, 0.05, restart=4, max_gmres_it=4, tol_gmres=1e-3, jv_mode=1, **kw)
    Ug = U.clone()
    sg = ctx.esdirk_step(Ug, 0.05, gmres=dict(restart=4, max_iter=4, tol=1e-3, jv_mode=frx.FR_JV_FD), **kw)
    print("forced halving", sg, so)
    assert so["halvings"] > 0
    assert sg["halvings"] == so["halvings"] and sg["ptc_iterations"] == so["ptc_iterations"]
    assert sg["status"] == so["status"] == 0
    err = np.linalg.norm(Ug.cpu().numpy() - Uo) / np.linalg.norm(Uo)
    print("rel diff", err)
    assert err <= 1e-7


@pytest.mark.parametrize("launch", ["per_bucket", "fused_2pass"])
def test_residual_parity_wall_32x32x8(frx, oracle_mod, launch):
    case = I.config(4)
    orc, ctx, U = _pair(frx, oracle_mod, case)
    ctx.set_launch(*LAUNCH[launch])
    R = ctx.residual(U)
    torch.cuda.synchronize()
    _full_size_residual_check(R.cpu().numpy(), orc, case, "c4 residual")


@pytest.mark.skip(reason="persistent (work-queue) launch mode withdrawn: its first GPU run faulted the GPU in the "
                         "dual-number Navier-Stokes fused tangent and no cause was shown; the mode is not built")
def test_persistent_queue_resets_across_calls_and_graph_replays(frx, c2):
    """The persistent launch resets its own work-queue counters: repeated
    calls and repeated graph-captured GMRES cycles give identical results."""
    case, orc, ctx, U = c2
    ctx.set_launch(True, persistent=True)
    R1 = ctx.residual(U).clone()
    for _ in range(3):
        assert torch.equal(ctx.residual(U), R1)
    ctx.set_launch(True, persistent=False)
    assert torch.equal(ctx.residual(U), R1)
    ctx.set_launch(True, persistent=True)
    F = torch.tensor(I.random_direction(case.U.size, 79).reshape(case.U.shape), device="cuda")
    xs = [ctx.gmres(U, 800.0, F, restart=6, max_iter=18, tol=0.0, use_graph=True)[0].clone() for _ in range(3)]
    assert torch.equal(xs[0], xs[1]) and torch.equal(xs[0], xs[2])


def test_nonphysical_flag(frx):
    case = CASES["vortex_p2_rusanov"]
    ctx = frx.Context.from_case(case)
    U = torch.tensor(case.U, device="cuda")
    U[0, 5] = -1.0
    ctx.residual(U)
    assert ctx.nonphysical() == 1
    assert ctx.nonphysical() == 0  # cleared by the read


def test_indicator_parity(frx, oracle_mod):
    for name in ("mixed_p1to5_ns_roe", "vortex_p2_rusanov", "wall_farfield_ns_roe"):
        case = CASES[name]
        orc, ctx, U = _pair(frx, oracle_mod, case)
        eta, mx = ctx.indicator(U, var=1)
        ref, rmx = orc.indicator(case.U, var=1)
        e = eta.cpu().numpy()
        assert np.max(np.abs(e - ref)) <= 1e-12 * max(1e-300, np.max(np.abs(ref)))
        assert abs(mx.item() - rmx) <= 1e-12 * rmx


def test_gmres_fixed_iterations_parity(frx, oracle_mod):
    case = CASES["mixed_p1to5_ns_roe"]
    orc, ctx, U = _pair(frx, oracle_mod, case, graphs=frx.FR_GRAPHS_ALL)
    F = I.random_direction(case.U.size, 77).reshape(case.U.shape)
    shift = 20.0
    xo, so = orc.gmres(case.U, shift, F, m=12, max_it=10, tol=0.0, jv_mode=0)
    for graph in (False, True):
        xg, sg = ctx.gmres(U, shift, torch.tensor(F, device="cuda"), restart=12, max_iter=10, tol=0.0,
                           use_graph=graph)
        assert sg["iterations"] == so["iterations"] == 10
        err = np.linalg.norm(xg.cpu().numpy() - xo) / np.linalg.norm(xo)
        print("gmres(10) rel diff", err, "graph", graph)
        assert err <= 1e-9
        assert abs(sg["rel_res"] - so["rel_res"]) <= 1e-9 * max(so["rel_res"], 1e-300) + 1e-12


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_gmres_one_pass_gram_schmidt_parity(frx, oracle_mod, prec):
    """One-pass classical Gram-Schmidt (FR_ORTHO_CGS, the PETSc default) spans
    the same Krylov space as the oracle's modified Gram-Schmidt: 10 fixed
    iterations of GMRES(30) (the fused Gram-Schmidt kernels up to 11 basis
    vectors) agree with the oracle, with and without the captured graphs, and
    match the CGS2 result of the same call."""
    case = CASES["mixed_p1to5_ns_roe"]
    orc, ctx, U = _pair(frx, oracle_mod, case, graphs=frx.FR_GRAPHS_ALL)
    F = I.random_direction(case.U.size, 79).reshape(case.U.shape)
    shift = 20.0
    p = frx.FR_F64 if prec == "f64" else frx.FR_F32
    xo, so = orc.gmres(case.U, shift, F, m=30, max_it=10, tol=0.0, jv_mode=0)
    Ft = torch.tensor(F, device="cuda")
    x2, s2 = ctx.gmres(U, shift, Ft, restart=30, max_iter=10, tol=0.0, precision=p)
    for graph in (False, True):
        xg, sg = ctx.gmres(U, shift, Ft, restart=30, max_iter=10, tol=0.0, use_graph=graph, precision=p,
                           orthog=frx.FR_ORTHO_CGS)
        assert sg["iterations"] == so["iterations"] == 10
        err = np.linalg.norm(xg.cpu().numpy() - xo) / np.linalg.norm(xo)
        d2 = (torch.linalg.norm(xg - x2) / torch.linalg.norm(x2)).item()
        print(prec, "CGS gmres(10) rel diff to oracle", err, "to CGS2", d2, "graph", graph, sg["rel_res"], so["rel_res"])
        assert err <= (1e-9 if p == frx.FR_F64 else 1e-4)
        assert d2 <= (1e-10 if p == frx.FR_F64 else 1e-4)


def test_gmres_one_pass_gram_schmidt_refusals(frx, oracle_mod):
    case = CASES["mixed_p1to5_ns_roe"]
    orc, ctx, U = _pair(frx, oracle_mod, case)
    for kw in (dict(restart=33, orthog=frx.FR_ORTHO_CGS), dict(restart=8, orthog=2)):
        with pytest.raises(frx.FrError) as ei:
            ctx.gmres(U, 10.0, U, **kw)
        assert ei.value.status == frx.FR_E_INVALID


def test_gmres_long_cycle_parity(frx, oracle_mod):
    """GMRES(40), 36 iterations in one cycle: the fused Gram-Schmidt kernels
    (up to 32 basis vectors) and the split multi-dot / multi-axpy path beyond
    them, against the oracle's modified Gram-Schmidt."""
    case = CASES["mixed_p1to5_ns_roe"]
    orc, ctx, U = _pair(frx, oracle_mod, case, graphs=frx.FR_GRAPHS_ALL)
    F = I.random_direction(case.U.size, 80).reshape(case.U.shape)
    shift = 8.0
    xo, so = orc.gmres(case.U, shift, F, m=40, max_it=36, tol=0.0, jv_mode=0)
    for graph in (False, True):
        xg, sg = ctx.gmres(U, shift, torch.tensor(F, device="cuda"), restart=40, max_iter=36, tol=0.0,
                           use_graph=graph)
        assert sg["iterations"] == so["iterations"] == 36
        err = np.linalg.norm(xg.cpu().numpy() - xo) / np.linalg.norm(xo)
        print("gmres(40) 36 its rel diff", err, "rel res", sg["rel_res"], so["rel_res"], "graph", graph)
        assert err <= 1e-8
        assert abs(sg["rel_res"] - so["rel_res"]) <= 1e-6 * so["rel_res"] + 1e-13


@pytest.mark.parametrize("mode", ["exact64", "fd64", "exact32", "exact64_graph", "exact32_graph"])
def test_gmres_converged(frx, oracle_mod, mode):
    case = CASES["wall_farfield_ns_roe"]
    orc, ctx, U = _pair(frx, oracle_mod, case, graphs=frx.FR_GRAPHS_ALL)
    F = I.random_direction(case.U.size, 78).reshape(case.U.shape)
    shift = 50.0  # (a shift of 5 makes GMRES(8) stagnate at 0.192 here, oracle and GPU alike)
    kw = dict(restart=8, max_iter=400, tol=1e-6, use_graph="graph" in mode,
              jv_mode=frx.FR_JV_FD if mode.startswith("fd") else frx.FR_JV_EXACT,
              precision=frx.FR_F32 if "32" in mode else frx.FR_F64)
    xg, sg = ctx.gmres(U, shift, torch.tensor(F, device="cuda"), **kw)
    assert sg["converged"], sg
    x = xg.cpu().numpy()
    # true residual with the oracle's exact operator
    r = F - (shift * x - orc.jvp(case.U, x))
    rel = np.linalg.norm(r) / np.linalg.norm(F)
    print(mode, sg, "true rel residual", rel)
    bound = 1e-5 if "32" in mode else 2e-6
    assert rel <= bound
    xo, so = orc.gmres(case.U, shift, F, m=8, max_it=400, tol=1e-6, jv_mode=0)
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 1e-4


def test_esdirk_stage_vortex_to_1e8(frx, oracle_mod):
    case = CASES["vortex_p2_rusanov"]
    orc, ctx, U = _pair(frx, oracle_mod, case)
    kw = dict(dtau_init=0.05, dtau_max=10.0, tol_pseudo=1e-8, last_stage=2)
    Uo, so = orc.esdirk2_step(case.U, 0.05, restart=20, tol_gmres=1e-8, jv_mode=1, **kw)
    Ug = U.clone()
    sg = ctx.esdirk_step(Ug, 0.05, gmres=dict(restart=20, tol=1e-8, jv_mode=frx.FR_JV_FD), **kw)
    print("stage", sg, so)
    assert sg["status"] == 0 and so["status"] == 0
    err = np.linalg.norm(Ug.cpu().numpy() - Uo) / np.linalg.norm(Uo)
    assert err <= 1e-7


def test_esdirk_full_step_mixed_vs_plain(frx, oracle_mod):
    case = CASES["mixed_p1to5_ns_roe"]
    orc, ctx, U = _pair(frx, oracle_mod, case, graphs=frx.FR_GRAPHS_ALL)
    kw = dict(dtau_init=0.005, dtau_max=0.05, tol_pseudo=1e-6)
    Uo, so = orc.esdirk2_step(case.U, 0.05, restart=30, tol_gmres=1e-3, jv_mode=0, **kw)
    ref = np.linalg.norm(Uo)
    for g in (dict(restart=30, tol=1e-3, jv_mode=frx.FR_JV_FD),
              dict(restart=30, tol=1e-3, jv_mode=frx.FR_JV_EXACT, precision=frx.FR_F32, use_graph=True),
              dict(restart=30, tol=1e-3, jv_mode=frx.FR_JV_EXACT, precision=frx.FR_F64, use_graph=True)):
        ctx.set_launch(g.get("use_graph", False))
        Ug = U.clone()
        sg = ctx.esdirk_step(Ug, 0.05, gmres=g, **kw)
        err = np.linalg.norm(Ug.cpu().numpy() - Uo) / ref
        print("full step", g, sg, "rel diff to oracle", err)
        assert sg["status"] == 0
        assert err <= 1e-6


@pytest.mark.parametrize("last_stage", [3, 5, 0], ids=["stage3", "stage5", "full"])
def test_esdirk4_vortex_to_1e8(frx, oracle_mod, last_stage):
    """ESDIRK4 (six stages): stage solutions and the full step on the vortex
    against the oracle's ESDIRK4, both solved to 1e-8."""
    case = CASES["vortex_p2_rusanov"]
    orc, ctx, U = _pair(frx, oracle_mod, case)
    kw = dict(dtau_init=0.05, dtau_max=10.0, tol_pseudo=1e-8, last_stage=last_stage)
    Uo, so = orc.esdirk_step(case.U, 0.1, restart=20, tol_gmres=1e-8, jv_mode=1, scheme=1, **kw)
    Ug = U.clone()
    sg = ctx.esdirk_step(Ug, 0.1, gmres=dict(restart=20, tol=1e-8, jv_mode=frx.FR_JV_FD), scheme=frx.FR_ESDIRK4,
                         **kw)
    print("ESDIRK4 last stage", last_stage, sg, so)
    assert sg["status"] == 0 and so["status"] == 0
    assert sg["stages"] == (5 if last_stage == 0 else last_stage - 1)
    err = np.linalg.norm(Ug.cpu().numpy() - Uo) / np.linalg.norm(Uo)
    print("rel diff", err)
    assert err <= 1e-7


def test_esdirk4_full_step_mixed_ns(frx, oracle_mod):
    """ESDIRK4 full step on mixed p = 1..5 Navier-Stokes: FP64 exact tangent
    with graphs and the mixed FP32 form against the oracle's ESDIRK4."""
    case = CASES["mixed_p1to5_ns_roe"]
    orc, ctx, U = _pair(frx, oracle_mod, case, graphs=frx.FR_GRAPHS_ALL)
    kw = dict(dtau_init=0.005, dtau_max=0.05, tol_pseudo=1e-6)
    Uo, so = orc.esdirk_step(case.U, 0.05, restart=30, tol_gmres=1e-3, jv_mode=0, scheme=1, **kw)
    assert so["status"] == 0
    ref = np.linalg.norm(Uo)
    ctx.set_launch(True)
    for g in (dict(restart=30, tol=1e-3, jv_mode=frx.FR_JV_EXACT, precision=frx.FR_F64, use_graph=True),
              dict(restart=30, tol=1e-3, jv_mode=frx.FR_JV_EXACT, precision=frx.FR_F32, use_graph=True)):
        Ug = U.clone()
        sg = ctx.esdirk_step(Ug, 0.05, gmres=g, scheme=frx.FR_ESDIRK4, **kw)
        err = np.linalg.norm(Ug.cpu().numpy() - Uo) / ref
        print("ESDIRK4 full step", g, sg, "rel diff to oracle", err)
        assert sg["status"] == 0 and sg["stages"] == 5
        assert err <= 1e-6


def test_esdirk_invalid_scheme_and_stage(frx, oracle_mod):
    case = CASES["vortex_p2_rusanov"]
    orc, ctx, U = _pair(frx, oracle_mod, case)
    for kw in (dict(scheme=2), dict(scheme=frx.FR_ESDIRK2, last_stage=4), dict(scheme=frx.FR_ESDIRK4, last_stage=7),
               dict(scheme=frx.FR_ESDIRK4, last_stage=1)):
        with pytest.raises(frx.FrError) as ei:
            ctx.esdirk_step(U.clone(), 0.05, dtau_init=0.05, dtau_max=1.0, **kw)
        assert ei.value.status == frx.FR_E_INVALID


def test_indicator_degree_field_matches_oracle(frx, oracle_mod):
    """The degree field of the vortex-street workload (at 16x16x2) chosen by
    the device (fr_select_degrees each sweep) equals the one the oracle's
    indicator, criteria and limiter choose (integer result: bit-exact)."""
    from oracle import degrees
    from paper_1910_03693_amd import adapt

    def make(ep):
        return I.case_street(16, 16, 2, elem_p=ep)

    p_gpu, hist = adapt.indicator_degree_field(make)
    p, hist_o = degrees.indicator_degree_field(
        make, lambda case: oracle_mod.Oracle.from_case(case).indicator(case.U, var=1))
    print("degree histogram", np.bincount(p_gpu, minlength=6)[1:], hist, hist_o)
    assert np.array_equal(p_gpu.astype(np.int64), p)
    assert hist == hist_o
