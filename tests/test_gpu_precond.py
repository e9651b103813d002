"""The element-Jacobi preconditioner (section 2.3) on the GPU against the
oracle: blocks built by coloured exact tangent products and LU-factored on the
device, applied to vectors (P^{-1} x against the oracle's dense solves of its
Jacobian blocks), GMRES with left preconditioning (fixed iterations: same
Krylov space as the oracle's preconditioned GMRES; converged: true residual),
and a preconditioned implicit stage against the oracle's stage solution."""
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


def _case(k=81, wall=True):
    return I.case_ns_mixed(3, 2, 2, k=k, lengths=(1.0, 0.7, 0.6), pvals=(1, 2, 3), pw=(1, 1, 1), re=200.0, ma=0.3,
                           wall=wall)


@pytest.fixture(scope="module")
def small(oracle_mod):
    from oracle import precond as PC
    case = _case()
    orc = oracle_mod.Oracle.from_case(case)
    J = orc.jacobian(case.U)
    dofs = PC.element_dofs(I.sp_offsets(case.elem_p), orc.n_sp)
    return case, orc, J, dofs


def _reserve(frx, prec):
    return frx.FR_RESERVE_PRECOND_F64 if prec == frx.FR_F64 else frx.FR_RESERVE_PRECOND_F32


def _prec(frx, name):
    return {"f64": frx.FR_F64, "f32": frx.FR_F32, "f16": frx.FR_PC_F16}[name]


# P^-1 x against the oracle's dense solves: float64 blocks, float32 blocks,
# and the float16 copy of sigma times the float32 inverse (11-bit significand)
APPLY_TOL = {"f64": 1e-11, "f32": 2e-4, "f16": 3e-3}


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
@pytest.mark.parametrize("fused", [True, False], ids=["fused", "per_bucket"])
def test_precond_apply_matches_oracle(frx, small, prec, fused):
    from oracle import precond as PC
    case, orc, J, dofs = small
    p = _prec(frx, prec)
    ctx = frx.Context.from_case(case, max_restart=10, graphs=_reserve(frx, p), fused=fused)
    U = torch.tensor(case.U, device="cuda")
    sigma = 35.0  # partial pivoting swaps 8-145 rows of each of these blocks (orders 40-320)
    ctx.precond_build(U, sigma, p)
    x = I.random_direction(case.U.size, 4081).reshape(case.U.shape)
    y = ctx.precond_apply(torch.tensor(x, device="cuda")).cpu().numpy().ravel()
    ref = PC.apply(PC.element_blocks(J, dofs, sigma), dofs, x.ravel())
    err = np.abs(y - ref).max() / np.abs(ref).max()
    print(prec, "fused" if fused else "per-bucket", "P^-1 x rel err", err)
    assert err <= APPLY_TOL[prec]


@pytest.fixture(scope="module")
def largest(oracle_mod):
    """Blocks of the largest orders: one element of p = 5 (N = 1080, the
    maximum) and one of p = 4 (N = 625, a ragged last panel in both
    precisions), six of p = 1."""
    from oracle import precond as PC
    case = I.case_ns_mixed(2, 2, 2, k=91, lengths=(1.0, 0.7, 0.6), pvals=(1, 4, 5), pw=(6, 1, 1), re=200.0, ma=0.3,
                           wall=True)
    assert sorted(set(int(q) for q in case.elem_p)) == [1, 4, 5]
    orc = oracle_mod.Oracle.from_case(case)
    J = orc.jacobian(case.U)
    dofs = PC.element_dofs(I.sp_offsets(case.elem_p), orc.n_sp)
    return case, J, dofs


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_precond_apply_largest_blocks(frx, largest, prec):
    from oracle import precond as PC
    case, J, dofs = largest
    p = _prec(frx, prec)
    ctx = frx.Context.from_case(case, max_restart=4, graphs=_reserve(frx, p), fused=True)
    U = torch.tensor(case.U, device="cuda")
    sigma = 60.0
    ctx.precond_build(U, sigma, p)
    x = I.random_direction(case.U.size, 4084).reshape(case.U.shape)
    y = ctx.precond_apply(torch.tensor(x, device="cuda")).cpu().numpy().ravel()
    ref = PC.apply(PC.element_blocks(J, dofs, sigma), dofs, x.ravel())
    err = np.abs(y - ref).max() / np.abs(ref).max()
    print(prec, "p = 1, 4, 5: P^-1 x rel err", err)
    assert err <= APPLY_TOL[prec]


@pytest.mark.parametrize("graph", [False, True])
def test_preconditioned_gmres_fixed_iterations_parity(frx, small, graph):
    from oracle import precond as PC
    case, orc, J, dofs = small
    ctx = frx.Context.from_case(case, max_restart=12, graphs=frx.FR_GRAPHS_F64_EXACT | frx.FR_RESERVE_PRECOND_F64,
                                fused=True)
    U = torch.tensor(case.U, device="cuda")
    shift = 20.0
    ctx.precond_build(U, shift)
    F = I.random_direction(case.U.size, 4082)
    xg, sg = ctx.gmres(U, shift, torch.tensor(F.reshape(case.U.shape), device="cuda"), restart=12, max_iter=10,
                       tol=0.0, use_graph=graph, precond=True)
    A = shift * np.eye(J.shape[0]) - J
    blocks = PC.element_blocks(J, dofs, shift)
    xo, its, rr = PC.gmres_left(lambda v: A @ v, lambda v: PC.apply(blocks, dofs, v), F, 12, 10, 0.0)
    err = np.linalg.norm(xg.cpu().numpy().ravel() - xo) / np.linalg.norm(xo)
    print("preconditioned GMRES(10) rel diff", err, sg, its, rr)
    assert sg["iterations"] == its == 10
    assert err <= 1e-9
    assert abs(sg["rel_res"] - rr) <= 1e-8 * rr + 1e-14


@pytest.mark.parametrize("prec", ["f64", "f32_graph", "f16_graph"])
def test_preconditioned_gmres_converges_with_fewer_products(frx, small, prec):
    case, orc, J, dofs = small
    p = frx.FR_F64 if prec == "f64" else frx.FR_F32
    ctx = frx.Context.from_case(case, max_restart=10,
                                graphs=_reserve(frx, p) | frx.FR_GRAPHS_F64_EXACT | frx.FR_GRAPHS_F32_EXACT,
                                fused=True)
    U = torch.tensor(case.U, device="cuda")
    shift = 8.0
    ctx.precond_build(U, shift, frx.FR_PC_F16 if prec.startswith("f16") else p)
    F = I.random_direction(case.U.size, 4083).reshape(case.U.shape)
    Ft = torch.tensor(F, device="cuda")
    kw = dict(restart=10, max_iter=600, tol=1e-6, precision=p, use_graph="graph" in prec)
    xp, sp = ctx.gmres(U, shift, Ft, precond=2 if prec.startswith("f16") else 1, **kw)
    x0, s0 = ctx.gmres(U, shift, Ft, precond=False, **kw)
    A = shift * np.eye(J.shape[0]) - J
    rel = np.linalg.norm(F.ravel() - A @ xp.cpu().numpy().ravel()) / np.linalg.norm(F)
    print(prec, "preconditioned", sp, "plain", s0, "true rel residual", rel)
    assert sp["converged"] and s0["converged"]
    assert sp["iterations"] < s0["iterations"]
    assert rel <= (1e-4 if p == frx.FR_F64 else 1e-3)


def test_preconditioned_stage_matches_oracle_stage(frx, oracle_mod):
    """One implicit ESDIRK2 stage solved to 1e-8 with the preconditioner built
    at the start of the step: the same stage solution as the oracle's
    (unpreconditioned) stage, since both solve the same stage equation."""
    case = I.config(1)
    orc = oracle_mod.Oracle.from_case(case)
    kw = dict(dtau_init=0.05, dtau_max=10.0, tol_pseudo=1e-8, last_stage=2)
    Uo, so = orc.esdirk2_step(case.U, 0.05, restart=20, tol_gmres=1e-8, jv_mode=0, **kw)
    ctx = frx.Context.from_case(case, max_restart=20, graphs=frx.FR_GRAPHS_F64_EXACT | frx.FR_RESERVE_PRECOND_F64,
                                fused=True)
    Ug = torch.tensor(case.U, device="cuda")
    sg = ctx.esdirk_step(Ug, 0.05, gmres=dict(restart=20, tol=1e-8, use_graph=True, precond=True), **kw)
    Up = torch.tensor(case.U, device="cuda")
    sp = ctx.esdirk_step(Up, 0.05, gmres=dict(restart=20, tol=1e-8, use_graph=True), **kw)
    err = np.linalg.norm(Ug.cpu().numpy() - Uo) / np.linalg.norm(Uo)
    print("preconditioned stage", sg, "plain stage", sp, "oracle", so, "rel diff", err)
    assert sg["status"] == 0 and so["status"] == 0
    assert err <= 1e-7
    assert sg["gmres_iterations"] < sp["gmres_iterations"]


def test_precond_refusals(frx):
    case = _case(83)
    ctx = frx.Context.from_case(case, max_restart=8)
    U = torch.tensor(case.U, device="cuda")
    for call in (lambda: ctx.precond_build(U, 10.0),                       # no storage reserved
                 lambda: ctx.precond_apply(U),                              # nothing built
                 lambda: ctx.gmres(U, 10.0, U, restart=8, precond=True)):   # nothing built
        with pytest.raises(frx.FrError) as ei:
            call()
        assert ei.value.status == frx.FR_E_INVALID
    ctx.reserve(8, frx.FR_RESERVE_PRECOND_F32)
    with pytest.raises(frx.FrError) as ei:
        ctx.precond_build(U, 10.0, frx.FR_F64)  # storage is float32
    assert ei.value.status == frx.FR_E_INVALID
    with pytest.raises(frx.FrError) as ei:
        ctx.precond_build(U, -1.0, frx.FR_F32)
    assert ei.value.status == frx.FR_E_INVALID
    ctx.precond_build(U, 10.0, frx.FR_F32)
    with pytest.raises(frx.FrError) as ei:
        ctx.gmres(U, 10.0, U, restart=8, precision=frx.FR_F32, precond=2)  # built without the float16 copy
    assert ei.value.status == frx.FR_E_INVALID
    ctx.precond_build(U, 10.0, frx.FR_PC_F16)
    with pytest.raises(frx.FrError) as ei:
        ctx.gmres(U, 10.0, U, restart=8, precision=frx.FR_F32, precond=1)  # built as float16
    assert ei.value.status == frx.FR_E_INVALID
    ctx2 = frx.Context.from_case(case, max_restart=8, graphs=frx.FR_RESERVE_PRECOND_F64)
    with pytest.raises(frx.FrError) as ei:
        ctx2.precond_build(U, 10.0, frx.FR_PC_F16)  # float16 needs float32 storage
    assert ei.value.status == frx.FR_E_INVALID
