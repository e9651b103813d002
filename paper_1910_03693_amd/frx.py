"""Python binding of libfrx.so (include/fr.h): argument marshalling only.

The module-level functions carry the C-ABI names and take torch tensors that
already live on the GPU; every step of the hot path runs in the HIP library.
PyTorch supplies device memory and the current stream.  If the library is not
built the binding raises; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfrx.so")

FR_OK, FR_E_INVALID, FR_E_NOMEM, FR_E_HIP, FR_E_NOTCONVERGED, FR_E_NONPHYSICAL, FR_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
FR_EULER, FR_NAVIER_STOKES = 0, 1
FR_ROE, FR_RUSANOV = 0, 1
FR_F64, FR_F32 = 0, 1
FR_JV_EXACT, FR_JV_FD, FR_JV_FD_SCALED = 0, 1, 2
FR_GRAPHS_F64_EXACT, FR_GRAPHS_F32_EXACT, FR_GRAPHS_F64_FD, FR_GRAPHS_F64_FD_SCALED, FR_GRAPHS_ALL = 1, 2, 4, 8, 15
FR_RESERVE_PRECOND_F64, FR_RESERVE_PRECOND_F32 = 16, 32
FR_LAUNCH_PER_BUCKET, FR_LAUNCH_FUSED = 0, 1
FR_LAUNCH_FACES_TWO_PASS, FR_LAUNCH_FACES_ONE_PASS = 4, 8
FR_ESDIRK2, FR_ESDIRK4 = 0, 1
FR_ETA_MAX_ALL, FR_ETA_MAX_SAME_DEGREE = 0, 1
FR_ORTHO_CGS2, FR_ORTHO_CGS = 0, 1
FR_PC_F16 = 2
STATUS_NAMES = {0: "FR_OK", -1: "FR_E_INVALID", -2: "FR_E_NOMEM", -3: "FR_E_HIP", -4: "FR_E_NOTCONVERGED",
                -5: "FR_E_NONPHYSICAL", -6: "FR_E_UNSUPPORTED"}
EXPORTED = ("fr_create", "fr_destroy", "fr_layout", "fr_reserve", "fr_residual", "fr_residual_noalloc", "fr_residual_jvp", "fr_jvp", "fr_vjp", "gmres_stage_solve",
            "esdirk_step", "spectral_decay_indicator", "fr_select_degrees", "fr_project", "fr_filter", "fr_autotune", "fr_profile",
            "fr_set_launch", "fr_check", "fr_launch_shapes", "fr_precond_build", "fr_precond_apply",
            "fr_trim", "fr_last_error")


class FrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class fr_mesh_desc(C.Structure):
    _fields_ = [("n_elem", C.c_int32), ("elem_xyz", C.POINTER(C.c_double)), ("elem_nbr", C.POINTER(C.c_int32)),
                ("elem_p", C.POINTER(C.c_int8)), ("physics", C.c_int32), ("flux", C.c_int32),
                ("gamma", C.c_double), ("mu", C.c_double), ("prandtl", C.c_double), ("farfield", C.c_double * 5)]


class fr_gmres_opts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("max_iter", C.c_int32), ("tol", C.c_double), ("jv_mode", C.c_int32),
                ("precision", C.c_int32), ("fd_eps", C.c_double), ("use_graph", C.c_int32),
                ("precond", C.c_int32), ("orthog", C.c_int32)]


class fr_gmres_stats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("cycles", C.c_int32), ("rel_res", C.c_double),
                ("converged", C.c_int32)]


class fr_step_opts(C.Structure):
    _fields_ = [("dtau_init", C.c_double), ("dtau_max", C.c_double), ("dtau_min", C.c_double),
                ("tol_pseudo", C.c_double), ("max_ptc_iter", C.c_int32), ("last_stage", C.c_int32),
                ("gmres", fr_gmres_opts), ("scheme", C.c_int32)]


class fr_step_stats(C.Structure):
    _fields_ = [("ptc_iterations", C.c_int32), ("gmres_iterations", C.c_int32), ("halvings", C.c_int32),
                ("stages", C.c_int32), ("final_rel_F", C.c_double)]


class fr_kernel_time(C.Structure):
    _fields_ = [("stage", C.c_char * 16), ("n_lo", C.c_int32), ("n_hi", C.c_int32), ("units", C.c_int64),
                ("ms", C.c_double)]


_lib = None


def lib():
    """Load libfrx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1910_03693_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.fr_create.restype = C.c_int
        L.fr_create.argtypes = [C.POINTER(fr_mesh_desc), C.POINTER(vp)]
        L.fr_destroy.argtypes = [vp]
        L.fr_layout.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.fr_reserve.argtypes = [vp, C.c_int32, C.c_int32]
        L.fr_residual.argtypes = [vp, vp, vp, vp]
        L.fr_residual_noalloc.argtypes = [vp, vp, vp, vp]
        L.fr_jvp.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_int32, C.c_double, vp]
        L.fr_vjp.argtypes = [vp, vp, vp, vp, vp]
        L.fr_residual_jvp.argtypes = [vp, vp, vp, vp, vp, vp]
        L.gmres_stage_solve.argtypes = [vp, vp, C.c_double, vp, vp, C.POINTER(fr_gmres_opts),
                                        C.POINTER(fr_gmres_stats), vp]
        L.esdirk_step.argtypes = [vp, vp, C.c_double, C.POINTER(fr_step_opts), C.POINTER(fr_step_stats), vp]
        L.spectral_decay_indicator.argtypes = [vp, vp, C.c_int32, vp, vp, vp]
        L.fr_select_degrees.argtypes = [vp, vp, C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_int32, C.c_int32,
                                        vp, vp]
        L.fr_project.argtypes = [vp, vp, vp, vp, vp]
        L.fr_filter.argtypes = [vp, vp, vp, C.c_double, C.c_int32, vp]
        L.fr_autotune.argtypes = [vp, vp, vp]
        L.fr_check.argtypes = [vp, C.POINTER(C.c_int32), vp]
        L.fr_set_launch.argtypes = [vp, C.c_int32]
        L.fr_profile.argtypes = [vp, vp, C.c_int32, C.c_int32, C.POINTER(fr_kernel_time), C.c_int32,
                                 C.POINTER(C.c_int32), vp]
        L.fr_launch_shapes.argtypes = [vp, C.c_int32, vp, C.c_int32, C.POINTER(C.c_int32)]
        L.fr_precond_build.argtypes = [vp, vp, C.c_double, C.c_int32, vp]
        L.fr_precond_apply.argtypes = [vp, vp, vp, vp]
        L.fr_trim.argtypes = []
        L.fr_last_error.restype = C.c_char_p
        L.fr_last_error.argtypes = [vp]
        for name in EXPORTED:
            if name not in ("fr_last_error",):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _check(st, ctx=None):
    if st != FR_OK:
        msg = lib().fr_last_error(ctx)
        raise FrError(st, msg.decode() if msg else "")
    return st


# (n_dof, n_elem) of every live handle, recorded by fr_create: the wrappers
# refuse tensors of another context's size before anything is launched
_SIZES = {}


def _sizes(h):
    try:
        return _SIZES[h.value if isinstance(h, C.c_void_p) else h]
    except KeyError:
        raise ValueError("unknown or destroyed context handle") from None


def _ndof(h):
    return _sizes(h)[0]


def _dev(t, dtype, n=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"expected a contiguous {dtype} tensor, got {t.dtype}")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


# ------------------------------------------------------------ C-ABI wrappers
def fr_create(elem_xyz, elem_nbr, elem_p, physics=FR_EULER, flux=FR_RUSANOV, gamma=1.4, mu=0.0, prandtl=0.72,
              farfield=None):
    """Returns (handle, keepalive) for a host mesh description."""
    xyz = np.ascontiguousarray(elem_xyz, dtype=np.float64)
    nbr = np.ascontiguousarray(elem_nbr, dtype=np.int32)
    p = np.ascontiguousarray(elem_p, dtype=np.int8)
    d = fr_mesh_desc()
    d.n_elem = len(p)
    d.elem_xyz = xyz.ctypes.data_as(C.POINTER(C.c_double))
    d.elem_nbr = nbr.ctypes.data_as(C.POINTER(C.c_int32))
    d.elem_p = p.ctypes.data_as(C.POINTER(C.c_int8))
    d.physics, d.flux, d.gamma, d.mu, d.prandtl = physics, flux, gamma, mu, prandtl
    ff = np.zeros(5) if farfield is None else np.asarray(farfield, dtype=np.float64)
    for i in range(5):
        d.farfield[i] = float(ff[i])
    h = C.c_void_p()
    _check(lib().fr_create(C.byref(d), C.byref(h)))
    n = C.c_int64()
    _check(lib().fr_layout(h, C.byref(n), None), h)
    _SIZES[h.value] = (n.value, len(p))
    return h


def fr_destroy(h):
    _SIZES.pop(h.value if isinstance(h, C.c_void_p) else h, None)
    return lib().fr_destroy(h)


def fr_reserve(h, max_restart=40, graph_sets=FR_GRAPHS_ALL):
    return _check(lib().fr_reserve(h, int(max_restart), int(graph_sets)), h)


def fr_layout(h, n_elem):
    n = C.c_int64()
    off = np.zeros(n_elem + 1, dtype=np.int64)
    _check(lib().fr_layout(h, C.byref(n), off.ctypes.data_as(C.POINTER(C.c_int64))), h)
    return n.value, off


def fr_residual(h, U, R, stream=None):
    n = _ndof(h)
    return _check(lib().fr_residual(h, _dev(U, torch.float64, n), _dev(R, torch.float64, n), _stream(stream)), h)


def fr_residual_noalloc(h, U, R, stream=None):
    n = _ndof(h)
    return _check(lib().fr_residual_noalloc(h, _dev(U, torch.float64, n), _dev(R, torch.float64, n),
                                            _stream(stream)), h)


def fr_jvp(h, U, v, Jv, precision=FR_F64, jv_mode=FR_JV_EXACT, fd_eps=1e-6, stream=None):
    dt = torch.float64 if precision == FR_F64 else torch.float32
    n = _ndof(h)
    return _check(lib().fr_jvp(h, _dev(U, torch.float64, n), _dev(v, dt, n), _dev(Jv, dt, n),
                               precision, jv_mode, fd_eps, _stream(stream)), h)


def fr_vjp(h, U, w, JTw, stream=None):
    n = _ndof(h)
    return _check(lib().fr_vjp(h, _dev(U, torch.float64, n), _dev(w, torch.float64, n),
                               _dev(JTw, torch.float64, n), _stream(stream)), h)


def gmres_opts(restart=30, max_iter=100, tol=1e-1, jv_mode=FR_JV_EXACT, precision=FR_F64, fd_eps=1e-6,
               use_graph=False, precond=False, orthog=FR_ORTHO_CGS2):
    o = fr_gmres_opts()
    o.restart, o.max_iter, o.tol, o.jv_mode, o.precision, o.fd_eps, o.use_graph, o.precond, o.orthog = (
        restart, max_iter, tol, jv_mode, precision, fd_eps, int(bool(use_graph)), int(precond), int(orthog))
    return o


def gmres_stage_solve(h, U, shift, F, dU, opts, stream=None, check=True):
    st = fr_gmres_stats()
    n = _ndof(h)
    r = lib().gmres_stage_solve(h, _dev(U, torch.float64, n), float(shift), _dev(F, torch.float64, n),
                                _dev(dU, torch.float64, n), C.byref(opts), C.byref(st), _stream(stream))
    if check and r not in (FR_OK, FR_E_NOTCONVERGED):
        _check(r, h)
    return r, dict(iterations=st.iterations, cycles=st.cycles, rel_res=st.rel_res, converged=bool(st.converged))


def step_opts(dtau_init, dtau_max, dtau_min=None, tol_pseudo=1e-4, max_ptc_iter=200, last_stage=0, gmres=None,
              scheme=FR_ESDIRK2):
    """last_stage 0: the full step; 2..s-1: that stage's solution.  dtau_min
    defaults to dtau_init / 2^20 (at most 20 halvings below the start)."""
    if dtau_min is None:
        dtau_min = dtau_init / 2.0 ** 20
    o = fr_step_opts()
    o.dtau_init, o.dtau_max, o.dtau_min, o.tol_pseudo = dtau_init, dtau_max, dtau_min, tol_pseudo
    o.max_ptc_iter, o.last_stage, o.scheme = max_ptc_iter, last_stage, scheme
    o.gmres = gmres if gmres is not None else gmres_opts()
    return o


def esdirk_step(h, U, dt, opts, stream=None, check=True):
    st = fr_step_stats()
    r = lib().esdirk_step(h, _dev(U, torch.float64, _ndof(h)), float(dt), C.byref(opts), C.byref(st),
                          _stream(stream))
    if check and r not in (FR_OK, FR_E_NOTCONVERGED):
        _check(r, h)
    return r, dict(ptc_iterations=st.ptc_iterations, gmres_iterations=st.gmres_iterations, halvings=st.halvings,
                   stages=st.stages, final_rel_F=st.final_rel_F)


def spectral_decay_indicator(h, U, var, eta, eta_max, stream=None):
    n, ne = _sizes(h)
    return _check(lib().spectral_decay_indicator(h, _dev(U, torch.float64, n), var, _dev(eta, torch.float64, ne),
                                                 _dev(eta_max, torch.float64, 1), _stream(stream)), h)


def fr_residual_jvp(h, U, v, R, Jv, stream=None):
    n = _ndof(h)
    return _check(lib().fr_residual_jvp(h, _dev(U, torch.float64, n), _dev(v, torch.float64, n), _dev(R, torch.float64, n),
                                        _dev(Jv, torch.float64, n), _stream(stream)), h)


def fr_select_degrees(h, U, var, nu_max, nu_min, p_min, p_max, p_new, eta_max_scope=FR_ETA_MAX_ALL, stream=None):
    n, ne = _sizes(h)
    return _check(lib().fr_select_degrees(h, _dev(U, torch.float64, n), var, nu_max, nu_min, p_min, p_max,
                                          eta_max_scope, _dev(p_new, torch.int8, ne), _stream(stream)), h)


def fr_project(h_src, U_src, h_dst, U_dst, stream=None):
    return _check(lib().fr_project(h_src, _dev(U_src, torch.float64, _ndof(h_src)), h_dst,
                                   _dev(U_dst, torch.float64, _ndof(h_dst)), _stream(stream)), h_dst)


def fr_filter(h, U, U_out, alpha, p_from, stream=None):
    n = _ndof(h)
    return _check(lib().fr_filter(h, _dev(U, torch.float64, n), _dev(U_out, torch.float64, n), alpha, p_from,
                                  _stream(stream)), h)


def fr_autotune(h, U, stream=None):
    return _check(lib().fr_autotune(h, _dev(U, torch.float64, _ndof(h)), _stream(stream)), h)


def fr_profile(h, U, op=0, reps=10, stream=None):
    """Average duration of every kernel launch of one operator (0 residual,
    1 float64 tangent, 2 float32 tangent, 3 residual and float64 tangent in
    one pass), timed with HIP events."""
    buf = (fr_kernel_time * 128)()
    n = C.c_int32(0)
    _check(lib().fr_profile(h, _dev(U, torch.float64, _ndof(h)), op, reps, buf, 128, C.byref(n), _stream(stream)), h)
    return [dict(stage=buf[i].stage.decode(), n_lo=buf[i].n_lo, n_hi=buf[i].n_hi, units=buf[i].units,
                 ms=buf[i].ms) for i in range(n.value)]


def fr_launch_shapes(h, kind):
    """[(stage, code, items per tile)] of the fused plans of scalar kind
    0 (float64), 1 (float64 dual) or 2 (float32 dual)."""
    buf = np.zeros(3 * 256, dtype=np.int32)
    n = C.c_int32(0)
    _check(lib().fr_launch_shapes(h, int(kind), C.c_void_p(buf.ctypes.data), 256, C.byref(n)), h)
    return [tuple(int(x) for x in buf[3 * i:3 * i + 3]) for i in range(n.value)]


def fr_trim():
    """Frees the device blocks that destroyed contexts returned to the
    library's cache."""
    return lib().fr_trim()


def fr_precond_build(h, U, sigma, precision=FR_F64, stream=None):
    return _check(lib().fr_precond_build(h, _dev(U, torch.float64, _ndof(h)), float(sigma), int(precision),
                                         _stream(stream)), h)


def fr_precond_apply(h, x, y, stream=None):
    n = _ndof(h)
    return _check(lib().fr_precond_apply(h, _dev(x, torch.float64, n), _dev(y, torch.float64, n), _stream(stream)), h)


def fr_set_launch(h, mode):
    return _check(lib().fr_set_launch(h, mode), h)


def fr_check(h, stream=None):
    f = C.c_int32(0)
    _check(lib().fr_check(h, C.byref(f), _stream(stream)), h)
    return f.value


# ------------------------------------------------------------------- context
class Context:
    """A mesh on the GPU; methods take and return torch tensors shaped [5, n_sp].

    max_restart / graphs: the solver workspace and Arnoldi graph sets that
    fr_reserve makes at construction (max_restart=0 reserves nothing; the
    solver calls then refuse to run until reserve() is called); fused: the
    launch mode, set before the graphs are captured (None keeps the default)."""

    def __init__(self, elem_xyz, elem_nbr, elem_p, physics=FR_EULER, flux=FR_RUSANOV, gamma=1.4, mu=0.0,
                 prandtl=0.72, farfield=None, max_restart=40, graphs=0, fused=None):
        self.n_elem = len(elem_p)
        self.h = fr_create(elem_xyz, elem_nbr, elem_p, physics, flux, gamma, mu, prandtl, farfield)
        self.n_dof, self.sp_offset = fr_layout(self.h, self.n_elem)
        self.n_sp = self.n_dof // 5
        if fused is not None:  # before the graphs are captured
            self.set_launch(fused)
        if max_restart:
            fr_reserve(self.h, max_restart, graphs)

    @classmethod
    def from_case(cls, case, **kw):
        return cls(**case.desc(), **kw)

    def reserve(self, max_restart=40, graphs=FR_GRAPHS_ALL):
        fr_reserve(self.h, max_restart, graphs)

    def close(self):
        if getattr(self, "h", None):
            fr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def residual(self, U, out=None):
        out = torch.empty_like(U) if out is None else out
        fr_residual(self.h, U, out)
        return out

    def jvp(self, U, v, precision=FR_F64, jv_mode=FR_JV_EXACT, fd_eps=1e-6, out=None):
        out = torch.empty_like(v) if out is None else out
        fr_jvp(self.h, U, v, out, precision, jv_mode, fd_eps)
        return out

    def vjp(self, U, w, out=None):
        out = torch.empty_like(w) if out is None else out
        fr_vjp(self.h, U, w, out)
        return out

    def gmres(self, U, shift, F, out=None, **kw):
        out = torch.empty_like(F) if out is None else out
        r, st = gmres_stage_solve(self.h, U, shift, F, out, gmres_opts(**kw))
        st["status"] = r
        return out, st

    def esdirk_step(self, U, dt, gmres=None, **kw):
        r, st = esdirk_step(self.h, U, dt, step_opts(gmres=gmres_opts(**(gmres or {})), **kw))
        st["status"] = r
        return st

    def indicator(self, U, var=1):
        eta = torch.empty(self.n_elem, dtype=torch.float64, device=U.device)
        mx = torch.empty(1, dtype=torch.float64, device=U.device)
        spectral_decay_indicator(self.h, U, var, eta, mx)
        return eta, mx

    def residual_jvp(self, U, v, R=None, Jv=None):
        """(R(U), J(U) v) in float64 from one forward-mode pass."""
        R = torch.empty_like(U) if R is None else R
        Jv = torch.empty_like(U) if Jv is None else Jv
        fr_residual_jvp(self.h, U, v, R, Jv)
        return R, Jv

    def select_degrees(self, U, var=1, nu_max=0.1, nu_min=0.001, p_min=1, p_max=5, eta_max_scope=FR_ETA_MAX_ALL):
        """Device int8 tensor [n_elem] of the degrees chosen by the criteria
        and the face limiter of section 3.1."""
        p = torch.empty(self.n_elem, dtype=torch.int8, device=U.device)
        fr_select_degrees(self.h, U, var, nu_max, nu_min, p_min, p_max, p, eta_max_scope)
        return p

    def project_to(self, U, dst):
        """U (this context's layout) moved to the context `dst` (same mesh)."""
        out = torch.empty((5, dst.n_dof // 5), dtype=torch.float64, device=U.device)
        fr_project(self.h, U, dst.h, out)
        return out

    def nodal_filter(self, U, alpha=0.2, p_from=3, out=None):
        """Nodal polynomial filter (section 4.2): in every element of degree
        >= p_from, (1 - alpha) q + alpha (q projected onto degree p - 1).
        out may be U (in place); by default a new tensor."""
        out = torch.empty_like(U) if out is None else out
        fr_filter(self.h, U, out, alpha, p_from)
        return out

    def autotune(self, U):
        fr_autotune(self.h, U)

    def set_launch(self, fused, two_pass_faces=None):
        """fused: one launch per stage over all degrees (else one per bucket);
        two_pass_faces: True / False force the Navier-Stokes face stage into
        two kernels / one kernel, None keeps the current (autotuned) choice."""
        mode = FR_LAUNCH_FUSED if fused else FR_LAUNCH_PER_BUCKET
        if two_pass_faces is not None:
            mode |= FR_LAUNCH_FACES_TWO_PASS if two_pass_faces else FR_LAUNCH_FACES_ONE_PASS
        fr_set_launch(self.h, mode)

    def precond_build(self, U, sigma, precision=FR_F64):
        fr_precond_build(self.h, U, sigma, precision)

    def precond_apply(self, x, out=None):
        out = torch.empty_like(x) if out is None else out
        fr_precond_apply(self.h, x, out)
        return out

    def launch_shapes(self, kind=1):
        return fr_launch_shapes(self.h, kind)

    def profile(self, U, op=0, reps=10):
        return fr_profile(self.h, U, op, reps)

    def nonphysical(self):
        return fr_check(self.h)


class FRResidual(torch.autograd.Function):
    """R(U) with the exact adjoint (backward -> fr_vjp) and exact tangent
    (forward-mode jvp -> fr_jvp); ``fr`` is a Context."""

    @staticmethod
    def forward(U, fr):
        return fr.residual(U.contiguous())

    @staticmethod
    def setup_context(ctx, inputs, output):
        U, fr = inputs
        ctx.fr = fr
        ctx.save_for_backward(U)
        ctx.save_for_forward(U)

    @staticmethod
    def backward(ctx, grad):
        (U,) = ctx.saved_tensors
        return ctx.fr.vjp(U, grad.contiguous()), None

    @staticmethod
    def jvp(ctx, tU, _tfr):
        (U,) = ctx.saved_tensors
        return ctx.fr.jvp(U, tU.contiguous())


def residual(U, fr):
    return FRResidual.apply(U, fr)
