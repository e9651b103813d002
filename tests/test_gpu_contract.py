"""Calling conventions of the C ABI on the GPU: solver workspace made by
fr_reserve (no solver call allocates device memory afterwards), refused
options, the finite-difference step read at replay by captured graphs, and
the binding's refusal of tensors sized for another context."""
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


def _case(k=95):
    return I.case_ns_mixed(4, 4, 2, k=k, lengths=(1.0, 1.0, 0.5), wall=True, pvals=(1, 2, 3, 4),
                           pw=(1, 1, 1, 1), re=200.0, ma=0.3)


def _solves(frx, ctx, U, F, out):
    """Every solver call once: GMRES in each (mode, precision) with and without
    graphs, an ESDIRK2 and an ESDIRK4 step."""
    for g in (False, True):
        for kw in (dict(), dict(precision=frx.FR_F32), dict(jv_mode=frx.FR_JV_FD),
                   dict(jv_mode=frx.FR_JV_FD_SCALED)):
            ctx.gmres(U, 30.0, F, out=out, restart=12, max_iter=20, tol=1e-3, use_graph=g, **kw)
    Uw = out
    Uw.copy_(U)
    ctx.esdirk_step(Uw, 0.01, gmres=dict(restart=12, tol=1e-3, use_graph=True), dtau_init=1e-3,
                    dtau_max=1e-2, max_ptc_iter=6)
    Uw.copy_(U)
    ctx.esdirk_step(Uw, 0.01, gmres=dict(restart=12, tol=1e-3, use_graph=True, precision=frx.FR_F32),
                    dtau_init=1e-3, dtau_max=1e-2, max_ptc_iter=6, scheme=frx.FR_ESDIRK4)
    torch.cuda.synchronize()


def test_solver_calls_allocate_nothing_after_reserve(frx):
    case = _case()
    U = torch.tensor(case.U, device="cuda")
    F = torch.tensor(I.random_direction(case.U.size, 97).reshape(case.U.shape), device="cuda")
    out = torch.empty_like(U)
    # a first context loads every kernel and graph path of the library
    warm = frx.Context.from_case(case, max_restart=12, graphs=frx.FR_GRAPHS_ALL)
    _solves(frx, warm, U, F, out)
    warm.close()
    ctx = frx.Context.from_case(case, max_restart=12, graphs=frx.FR_GRAPHS_ALL)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    _solves(frx, ctx, U, F, out)
    free1, _ = torch.cuda.mem_get_info()
    print("free device memory before / after the first solver calls:", free0, free1)
    assert free1 == free0


def test_solver_options_beyond_the_reservation_are_refused(frx):
    case = _case()
    U = torch.tensor(case.U, device="cuda")
    F = torch.tensor(I.random_direction(case.U.size, 97).reshape(case.U.shape), device="cuda")
    ctx = frx.Context.from_case(case, max_restart=8, graphs=frx.FR_GRAPHS_F64_EXACT)
    with pytest.raises(frx.FrError) as ei:
        ctx.gmres(U, 30.0, F, restart=9)
    assert ei.value.status == frx.FR_E_INVALID
    with pytest.raises(frx.FrError) as ei:
        ctx.gmres(U, 30.0, F, restart=8, precision=frx.FR_F32, use_graph=True)
    assert ei.value.status == frx.FR_E_INVALID
    x, st = ctx.gmres(U, 30.0, F, restart=8, use_graph=True, tol=1e-2, max_iter=40)
    assert st["status"] in (frx.FR_OK, frx.FR_E_NOTCONVERGED)
    bare = frx.Context.from_case(case, max_restart=0)
    with pytest.raises(frx.FrError) as ei:
        bare.esdirk_step(U.clone(), 0.01, dtau_init=1e-3, dtau_max=1e-2)
    assert ei.value.status == frx.FR_E_INVALID
    with pytest.raises(frx.FrError) as ei:
        bare.gmres(U, 30.0, F, restart=4)
    assert ei.value.status == frx.FR_E_INVALID
    for kw in (dict(dtau_init=1e-3, dtau_max=1e-2, dtau_min=0.0), dict(dtau_init=1e-3, dtau_max=1e-4),
               dict(dtau_init=1e-3, dtau_max=1e-2, dtau_min=2e-3), dict(dtau_init=0.0, dtau_max=1e-2, dtau_min=0.0),
               dict(dtau_init=1e-3, dtau_max=1e-2, tol_pseudo=-1.0)):
        with pytest.raises(frx.FrError) as ei:
            ctx.esdirk_step(U.clone(), 0.01, gmres=dict(restart=8), **kw)
        assert ei.value.status == frx.FR_E_INVALID, kw
    with pytest.raises(frx.FrError) as ei:
        ctx.jvp(U, F, jv_mode=frx.FR_JV_FD, fd_eps=-1e-6)
    assert ei.value.status == frx.FR_E_INVALID


@pytest.mark.parametrize("mode", ["fd", "fd_scaled"])
def test_captured_graphs_read_the_current_fd_step(frx, mode):
    """Two GMRES solves with different finite-difference steps through the
    same captured graphs equal the same solves without graphs, bit for bit."""
    jv = frx.FR_JV_FD if mode == "fd" else frx.FR_JV_FD_SCALED
    case = _case(96)
    ctx = frx.Context.from_case(case, max_restart=10, graphs=frx.FR_GRAPHS_ALL)
    U = torch.tensor(case.U, device="cuda")
    F = torch.tensor(I.random_direction(case.U.size, 98).reshape(case.U.shape), device="cuda")
    res = {}
    for g in (True, False):
        for eps in (1e-6, 1e-4):
            x, st = ctx.gmres(U, 30.0, F, restart=10, max_iter=10, tol=0.0, jv_mode=jv, fd_eps=eps, use_graph=g)
            res[(g, eps)] = x.clone()
    for eps in (1e-6, 1e-4):
        assert torch.equal(res[(True, eps)], res[(False, eps)]), eps
    assert not torch.equal(res[(True, 1e-6)], res[(True, 1e-4)])


def test_tensors_of_another_context_are_refused_before_any_launch(frx):
    small = _case()
    other = I.case_ns_mixed(3, 3, 2, k=7, lengths=(1.0, 1.0, 0.5), pvals=(2, 3), pw=(1, 1))
    ctx = frx.Context.from_case(small, max_restart=4)
    Uo = torch.tensor(other.U, device="cuda")
    U = torch.tensor(small.U, device="cuda")
    assert Uo.numel() != U.numel()
    sentinel = torch.full_like(Uo, 7.0)
    calls = [lambda: frx.fr_residual(ctx.h, Uo, sentinel),
             lambda: frx.fr_jvp(ctx.h, Uo, Uo, sentinel),
             lambda: frx.fr_vjp(ctx.h, Uo, Uo, sentinel),
             lambda: frx.fr_residual_jvp(ctx.h, Uo, Uo, sentinel, torch.full_like(Uo, 7.0)),
             lambda: frx.fr_filter(ctx.h, Uo, sentinel, 0.2, 3),
             lambda: frx.gmres_stage_solve(ctx.h, Uo, 10.0, Uo, sentinel, frx.gmres_opts(restart=4)),
             lambda: frx.esdirk_step(ctx.h, sentinel, 0.01, frx.step_opts(1e-3, 1e-2)),
             lambda: frx.spectral_decay_indicator(ctx.h, Uo, 1, sentinel[0, :small.mesh["n_elem"]],
                                                  sentinel[1, :1]),
             lambda: frx.fr_residual(ctx.h, U, sentinel),
             lambda: frx.spectral_decay_indicator(ctx.h, U, 1, sentinel[0, :other.mesh["n_elem"]],
                                                  sentinel[1, :1])]
    for k, call in enumerate(calls):
        with pytest.raises(ValueError):
            call()
    torch.cuda.synchronize()
    assert torch.all(sentinel == 7.0)
