"""CPU oracle (test infrastructure only).

ctypes front end of ``fr_oracle.cpp``: a plain double-precision CPU reference of
the flux-reconstruction residual, its exact tangent (complex step), the finite-
difference product, dense Jacobians, restarted GMRES, pseudo-transient
continuation with ESDIRK2 and the spectral-decay indicator.  Only the tests,
the smoke check and the CPU-baseline leg of the benchmark use it; the product
library never loads it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "fr_oracle.cpp")


def build(force=True):
    """Compile the oracle with g++ (no GPU code, no shared source)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp",
                               "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        L.oracle_create.restype = C.c_void_p
        L.oracle_create.argtypes = [C.c_int, dp, ip, C.POINTER(C.c_int8), C.c_int, C.c_int,
                                    C.c_double, C.c_double, C.c_double, dp]
        L.oracle_destroy.argtypes = [C.c_void_p]
        L.oracle_nsp.restype = C.c_long
        L.oracle_nsp.argtypes = [C.c_void_p]
        for name in ("oracle_residual", "oracle_residual_ld"):
            getattr(L, name).argtypes = [C.c_void_p, dp, dp]
        L.oracle_residual_terms.argtypes = [C.c_void_p, dp, dp, dp]
        L.oracle_count_flops.restype = C.c_longlong
        L.oracle_count_flops.argtypes = [C.c_void_p, dp, dp, C.c_int, dp]
        L.oracle_threads.restype = C.c_int
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_jvp_cs.argtypes = [C.c_void_p, dp, dp, dp]
        L.oracle_jvp_fd.argtypes = [C.c_void_p, dp, dp, C.c_double, dp]
        L.oracle_jacobian.argtypes = [C.c_void_p, dp, dp]
        L.oracle_ops1d.argtypes = [C.c_int] + [dp] * 7
        L.oracle_radau_gL_d.restype = C.c_double
        L.oracle_radau_gL_d.argtypes = [C.c_int, C.c_double]
        L.oracle_interp_project.argtypes = [C.c_int, C.c_int, dp, dp]
        L.oracle_mass.argtypes = [C.c_void_p, dp]
        L.oracle_boundary_flux.argtypes = [C.c_void_p, dp, dp]
        L.oracle_indicator.argtypes = [C.c_void_p, dp, C.c_int, dp, dp]
        L.oracle_gmres.restype = C.c_int
        L.oracle_gmres.argtypes = [C.c_void_p, dp, C.c_double, dp, dp, C.c_int, C.c_int, C.c_double,
                                   C.c_int, C.c_double, ip, dp]
        L.oracle_esdirk2_step.restype = C.c_int
        L.oracle_esdirk2_step.argtypes = [C.c_void_p, dp, C.c_double, dp, dp]
        L.oracle_esdirk_step.restype = C.c_int
        L.oracle_esdirk_step.argtypes = [C.c_void_p, dp, C.c_double, dp, dp, C.c_int]
        L.oracle_esdirk_tableau.restype = C.c_int
        L.oracle_esdirk_tableau.argtypes = [C.c_int, dp, dp, dp]
        L.oracle_common_flux.argtypes = [C.c_int, C.c_double, dp, dp, dp, dp]
        L.oracle_physical_flux.argtypes = [C.c_double, C.c_double, C.c_double, dp, dp, dp]
        L.oracle_esdirk2_tableau.argtypes = [dp, dp, dp]
        L.oracle_physical_flux_n.argtypes = [C.c_long, C.c_double, C.c_double, C.c_double, dp, dp, dp]
        _lib = L
    return _lib


def threads():
    """Threads the oracle's OpenMP loops use (OMP_NUM_THREADS, else all cores)."""
    return int(lib().oracle_threads())


def set_threads(n):
    """Threads of the oracle's OpenMP loops from now on."""
    lib().oracle_set_threads(int(n))


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def ops1d(n):
    """Gauss nodes, weights, D, l(-1), l(+1), g_L'(x_k), g_R'(x_k) for n points."""
    x, w, lm, lp, gl, gr = (np.zeros(n) for _ in range(6))
    D = np.zeros((n, n))
    lib().oracle_ops1d(n, _p(x), _p(w), _p(D), _p(lm), _p(lp), _p(gl), _p(gr))
    return dict(x=x, w=w, D=D, lm=lm, lp=lp, gLp=gl, gRp=gr)


def common_flux(flux, qL, qR, S, gamma=1.4):
    out = np.zeros(5)
    lib().oracle_common_flux(flux, gamma, _p(_f64(qL)), _p(_f64(qR)), _p(_f64(S)), _p(out))
    return out


def physical_flux(q, G, gamma=1.4, mu=0.0, prandtl=0.72):
    """f[c, v] = inviscid - viscous flux in physical direction c."""
    f = np.zeros((3, 5))
    lib().oracle_physical_flux(gamma, mu, prandtl, _p(_f64(q)), _p(_f64(G)), _p(f))
    return f


def physical_flux_n(q, G, gamma=1.4, mu=0.0, prandtl=0.72):
    """q [npts, 5], G [npts, 5, 3] -> f [npts, 3, 5]."""
    q = _f64(q)
    G = _f64(G)
    f = np.zeros((q.shape[0], 3, 5))
    lib().oracle_physical_flux_n(q.shape[0], gamma, mu, prandtl, _p(q), _p(G), _p(f))
    return f


def esdirk2_tableau():
    A = np.zeros((3, 3))
    b = np.zeros(3)
    c = np.zeros(3)
    lib().oracle_esdirk2_tableau(_p(A), _p(b), _p(c))
    return A, b, c


def esdirk_tableau(scheme):
    """(A, b, c) of scheme 0 (ESDIRK2, 3 stages) or 1 (ESDIRK4, 6 stages)."""
    A = np.zeros(36)
    b = np.zeros(6)
    c = np.zeros(6)
    s = lib().oracle_esdirk_tableau(scheme, _p(A), _p(b), _p(c))
    if s == 0:
        raise ValueError(f"unknown ESDIRK scheme {scheme}")
    return A[:s * s].reshape(s, s).copy(), b[:s].copy(), c[:s].copy()


def radau_gL_d(p, x):
    return lib().oracle_radau_gL_d(p, x)


def interp_project(n_lo, n_hi):
    I = np.zeros((n_hi, n_lo))
    P = np.zeros((n_lo, n_hi))
    lib().oracle_interp_project(n_lo, n_hi, _p(I), _p(P))
    return I, P


class Oracle:
    """One mesh + physics description; arrays as in ``inputs`` (U is [5, n_sp])."""

    def __init__(self, elem_xyz, elem_nbr, elem_p, physics=0, flux=1, gamma=1.4, mu=0.0,
                 prandtl=0.72, farfield=None):
        self._xyz = _f64(elem_xyz)
        self._nbr = np.ascontiguousarray(elem_nbr, dtype=np.int32)
        self._p = np.ascontiguousarray(elem_p, dtype=np.int8)
        ff = _f64(np.zeros(5) if farfield is None else farfield)
        self._ff = ff
        L = lib()
        self.h = L.oracle_create(len(self._p), _p(self._xyz), self._nbr.ctypes.data_as(C.POINTER(C.c_int32)),
                                 self._p.ctypes.data_as(C.POINTER(C.c_int8)), physics, flux, gamma, mu,
                                 prandtl, _p(ff))
        if not self.h:
            raise ValueError("invalid mesh description")
        self.n_sp = L.oracle_nsp(self.h)
        self.shape = (5, self.n_sp)

    @classmethod
    def from_case(cls, case):
        return cls(**case.desc())

    def __del__(self):
        if getattr(self, "h", None):
            lib().oracle_destroy(self.h)
            self.h = None

    def _vec(self, a):
        a = _f64(a)
        assert a.size == 5 * self.n_sp
        return a

    def residual(self, U):
        U = self._vec(U)
        R = np.zeros(self.shape)
        lib().oracle_residual(self.h, _p(U), _p(R))
        return R

    def count_flops(self, U, v=None):
        """Floating-point operations of one residual evaluation at U (v None)
        or of one residual-and-tangent evaluation along v in forward-mode dual
        arithmetic, counted operation by operation on the oracle's own code
        (one per +, -, *, / and square root; the dual operations at their cost
        in that arithmetic).  Returns (flops, R or J v)."""
        U = self._vec(U)
        out = np.zeros_like(U)
        if v is None:
            f = lib().oracle_count_flops(self.h, _p(U), _p(U), 0, _p(out))
        else:
            v = self._vec(v)
            f = lib().oracle_count_flops(self.h, _p(U), _p(v), 1, _p(out))
        return int(f), out

    def residual_terms(self, U):
        """(R, T): the residual and, per solution point, the sum of the
        absolute values of the terms it adds up over |J|."""
        U = self._vec(U)
        R, T = np.zeros(self.shape), np.zeros(self.shape)
        lib().oracle_residual_terms(self.h, _p(U), _p(R), _p(T))
        return R, T

    def residual_ld(self, U):
        """The residual evaluated in extended precision (rounding reference)."""
        U = self._vec(U)
        R = np.zeros(self.shape)
        lib().oracle_residual_ld(self.h, _p(U), _p(R))
        return R

    def jvp(self, U, v):
        """Exact tangent by the complex step."""
        U, v = self._vec(U), self._vec(v)
        out = np.zeros(self.shape)
        lib().oracle_jvp_cs(self.h, _p(U), _p(v), _p(out))
        return out

    def jvp_fd(self, U, v, eps=1e-6):
        U, v = self._vec(U), self._vec(v)
        out = np.zeros(self.shape)
        lib().oracle_jvp_fd(self.h, _p(U), _p(v), eps, _p(out))
        return out

    def jacobian(self, U):
        U = self._vec(U)
        n = 5 * self.n_sp
        J = np.zeros((n, n))
        lib().oracle_jacobian(self.h, _p(U), _p(J))
        return J

    def mass(self):
        """w_i w_j w_k J at every solution point, [n_sp]."""
        m = np.zeros(self.n_sp)
        lib().oracle_mass(self.h, _p(m))
        return m

    def boundary_flux(self, U):
        U = self._vec(U)
        out = np.zeros(5)
        lib().oracle_boundary_flux(self.h, _p(U), _p(out))
        return out

    def indicator(self, U, var=1):
        U = self._vec(U)
        eta = np.zeros(len(self._p))
        mx = np.zeros(1)
        lib().oracle_indicator(self.h, _p(U), var, _p(eta), _p(mx))
        return eta, float(mx[0])

    def gmres(self, U, shift, F, m=30, max_it=100, tol=1e-1, jv_mode=0, fd_eps=1e-6):
        U, F = self._vec(U), self._vec(F)
        x = np.zeros(self.shape)
        its = C.c_int32(0)
        rr = np.zeros(1)
        st = lib().oracle_gmres(self.h, _p(U), shift, _p(F), _p(x), m, max_it, tol, jv_mode, fd_eps,
                                C.byref(its), _p(rr))
        return x, dict(status=st, iterations=its.value, rel_res=float(rr[0]))

    def esdirk2_step(self, U, dt, dtau_init, dtau_max, dtau_min=0.0, tol_pseudo=1e-4, tol_gmres=1e-1,
                     restart=60, max_gmres_it=100, max_ptc_it=200, jv_mode=1, fd_eps=1e-6, last_stage=3):
        return self.esdirk_step(U, dt, dtau_init, dtau_max, dtau_min, tol_pseudo, tol_gmres, restart, max_gmres_it,
                                max_ptc_it, jv_mode, fd_eps, last_stage, scheme=0)

    def esdirk_step(self, U, dt, dtau_init, dtau_max, dtau_min=0.0, tol_pseudo=1e-4, tol_gmres=1e-1,
                    restart=60, max_gmres_it=100, max_ptc_it=200, jv_mode=1, fd_eps=1e-6, last_stage=0, scheme=0):
        """One step of scheme 0 (ESDIRK2) or 1 (ESDIRK4); last_stage 0 (or the
        stage count) for the full step, 2..s-1 for a stage solution."""
        Uo = self._vec(U).copy()
        opts = _f64([dtau_init, dtau_max, dtau_min, tol_pseudo, tol_gmres, restart, max_gmres_it,
                     max_ptc_it, jv_mode, fd_eps, last_stage])
        stats = np.zeros(4)
        st = lib().oracle_esdirk_step(self.h, _p(Uo), dt, _p(opts), _p(stats), scheme)
        return Uo, dict(status=st, ptc_iterations=int(stats[0]), gmres_iterations=int(stats[1]),
                        halvings=int(stats[2]), final_rel_F=float(stats[3]))
