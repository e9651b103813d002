"""Seeded synthetic inputs: hexahedral box meshes, per-element degree fields and
analytic flow fields sampled at the solution points.

This module defines *inputs only*.  It holds none of the flux-reconstruction
arithmetic (no operators, fluxes, residuals or solvers); both the HIP library and
the CPU oracle receive exactly the arrays built here.  Solution points are the
tensor Gauss-Legendre points of each element (numpy's ``leggauss``) mapped through
the element's trilinear vertex map, which is how the initial condition is
defined: the nodal interpolant of an analytic field at the solution points.

Mesh arrays (all numpy, C order):
  ``elem_xyz`` float64 [E, 8, 3]  vertex v = a + 2b + 4c sits at reference
                                   (xi, eta, zeta) = (2a-1, 2b-1, 2c-1)
  ``elem_nbr`` int32   [E, 6]     faces (-xi, +xi, -eta, +eta, -zeta, +zeta):
                                   neighbour element id, or -1 (no-slip adiabatic
                                   wall) / -2 (far field)
  ``elem_p``   int8    [E]        polynomial degree 1..5
State layout: ``U[var, sp]`` with var = (rho, rho u, rho v, rho w, rho E), each
element's (p+1)^3 block contiguous in element order, xi index fastest.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 1.4
BC_WALL = -1
BC_FARFIELD = -2


# --------------------------------------------------------------------------- mesh
def box_mesh(nx, ny, nz, lengths, periodic=(True, True, True), noise=0.0,
             seed=None, origin=(0.0, 0.0, 0.0), bc_lo=None, bc_hi=None):
    """Structured box of nx*ny*nz hexahedra, element e = ix + nx*(iy + ny*iz).

    ``noise`` is the standard deviation of the Gaussian vertex displacement (per
    coordinate, absolute units).  Periodic images of a vertex move together; in a
    non-periodic direction the vertices on the two boundary planes do not move.
    ``bc_lo[d]``/``bc_hi[d]`` give the boundary code on the low/high side of a
    non-periodic direction d.
    """
    nn = (nx, ny, nz)
    L = np.asarray(lengths, dtype=np.float64)
    h = L / np.asarray(nn, dtype=np.float64)
    # unique vertex lattice: a periodic direction has n unique planes, else n+1
    nu = [nn[d] if periodic[d] else nn[d] + 1 for d in range(3)]
    disp = np.zeros((nu[0], nu[1], nu[2], 3))
    if noise > 0.0:
        rng = np.random.default_rng(seed)
        disp = rng.normal(0.0, noise, size=disp.shape)
        for d in range(3):
            if not periodic[d]:
                sl = [slice(None)] * 3
                sl[d] = 0
                disp[tuple(sl)] = 0.0
                sl[d] = nu[d] - 1
                disp[tuple(sl)] = 0.0

    E = nx * ny * nz
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ijk = [ix.ravel(), iy.ravel(), iz.ravel()]  # element e = ix + nx (iy + ny iz)
    elem_xyz = np.zeros((E, 8, 3))
    for c in range(2):
        for b in range(2):
            for a in range(2):
                idx = [ijk[0] + a, ijk[1] + b, ijk[2] + c]
                # a periodic image (index n) takes the displacement of plane 0
                u = [idx[d] % nn[d] if periodic[d] else idx[d] for d in range(3)]
                base = np.asarray(origin)[None, :] + np.stack(idx, axis=1).astype(np.float64) * h[None, :]
                elem_xyz[:, a + 2 * b + 4 * c] = base + disp[u[0], u[1], u[2]]
    elem_nbr = np.zeros((E, 6), dtype=np.int32)
    bc_lo = bc_lo or [BC_WALL] * 3
    bc_hi = bc_hi or [BC_WALL] * 3
    for d in range(3):
        for s in range(2):
            j = [q.copy() for q in ijk]
            j[d] = j[d] + (1 if s else -1)
            inside = (j[d] >= 0) & (j[d] < nn[d])
            j[d] = j[d] % nn[d]
            nb = j[0] + nx * (j[1] + ny * j[2])
            if not periodic[d]:
                nb = np.where(inside, nb, bc_hi[d] if s else bc_lo[d])
            elem_nbr[:, 2 * d + s] = nb
    return {"elem_xyz": elem_xyz, "elem_nbr": elem_nbr, "n_elem": E,
            "shape": nn, "lengths": tuple(L), "periodic": tuple(periodic)}


def draw_p(n_elem, values, weights, seed):
    """i.i.d. per-element degrees drawn with numpy default_rng(seed)."""
    rng = np.random.default_rng(seed)
    w = np.asarray(weights, dtype=np.float64)
    return rng.choice(np.asarray(values, dtype=np.int8), size=n_elem, p=w / w.sum()).astype(np.int8)


def sp_offsets(elem_p):
    n3 = (np.asarray(elem_p, dtype=np.int64) + 1) ** 3
    off = np.zeros(len(n3) + 1, dtype=np.int64)
    np.cumsum(n3, out=off[1:])
    return off


def solution_points(mesh, elem_p):
    """Physical coordinates [3, n_sp] of every solution point (input definition)."""
    xyz = mesh["elem_xyz"]
    elem_p = np.asarray(elem_p)
    off = sp_offsets(elem_p)
    out = np.zeros((3, off[-1]))
    for p in np.unique(elem_p):
        n = int(p) + 1
        x1, _ = np.polynomial.legendre.leggauss(n)
        # tensor points, xi fastest
        Z, Y, X = np.meshgrid(x1, x1, x1, indexing="ij")
        xi, eta, zeta = X.ravel(), Y.ravel(), Z.ravel()
        N = np.zeros((n ** 3, 8))
        for c in range(2):
            for b in range(2):
                for a in range(2):
                    N[:, a + 2 * b + 4 * c] = 0.125 * (1 + (2 * a - 1) * xi) * \
                        (1 + (2 * b - 1) * eta) * (1 + (2 * c - 1) * zeta)
        els = np.nonzero(elem_p == p)[0]
        pts = np.einsum("kv,evc->eck", N, xyz[els])  # [e, 3, n^3]
        idx = off[els][:, None] + np.arange(n ** 3)[None, :]
        for c in range(3):
            out[c, idx] = pts[:, c, :]
    return out


# ------------------------------------------------------------------- flow fields
def primitive_to_conservative(rho, u, v, w, p, gamma=GAMMA):
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E])


def vortex_field(x, y, z, x0, y0, t=0.0, ma=0.5, uinf=(1.0, 0.0, 0.0),
                 alpha=5.0, phi=0.5, gamma=GAMMA, period=None):
    """Isentropic vortex (section 3.3 of the paper, the fluctuation equations),
    freestream rho = 1, |u| from ``uinf``, p = 1/(gamma Ma^2), gas constant 1.
    The centre translates with the freestream; ``period`` (Lx, Ly) wraps it."""
    cx = x0 + uinf[0] * t
    cy = y0 + uinf[1] * t
    dx = x - cx
    dy = y - cy
    if period is not None:
        dx = (dx + 0.5 * period[0]) % period[0] - 0.5 * period[0]
        dy = (dy + 0.5 * period[1]) % period[1] - 0.5 * period[1]
    r2 = dx * dx + dy * dy
    ex = np.exp(phi * (1.0 - r2))
    du = -alpha / (2 * math.pi) * dy * ex
    dv = alpha / (2 * math.pi) * dx * ex
    tinf = 1.0 / (gamma * ma * ma)
    dT = -alpha ** 2 * (gamma - 1.0) / (16.0 * phi * gamma * math.pi ** 2) * ex * ex
    T = tinf + dT
    rho = (T / tinf) ** (1.0 / (gamma - 1.0))
    p = rho * T
    return primitive_to_conservative(rho, uinf[0] + du, uinf[1] + dv, uinf[2] + 0 * x, p, gamma)


@dataclass
class FourierModes:
    """Divergence-free velocity u' = sum_k Re(a_k exp(i k.x)), a_k orthogonal to k,
    k = 2 pi (mx/Lx, my/Ly, mz/Lz), 0 < |k| <= kmax, scaled to max|u'| = amp on a
    fixed lattice of the domain."""
    lengths: tuple
    kmax: float
    amp: float
    seed: int
    m: np.ndarray = field(init=False)
    a: np.ndarray = field(init=False)

    def __post_init__(self):
        Lx, Ly, Lz = self.lengths
        mr = [int(math.floor(self.kmax * Ld / (2 * math.pi) + 1e-9)) for Ld in self.lengths]
        ms = []
        for mz in range(-mr[2], mr[2] + 1):
            for my in range(-mr[1], mr[1] + 1):
                for mx in range(-mr[0], mr[0] + 1):
                    k = 2 * math.pi * np.array([mx / Lx, my / Ly, mz / Lz])
                    kn = np.linalg.norm(k)
                    if 0 < kn <= self.kmax * (1 + 1e-12):
                        ms.append((mx, my, mz))
        self.m = np.asarray(ms, dtype=np.float64)
        rng = np.random.default_rng(self.seed)
        a = rng.normal(size=(len(ms), 3)) + 1j * rng.normal(size=(len(ms), 3))
        k = self.kvec()
        kk = np.sum(k * k, axis=1, keepdims=True)
        a = a - k * (np.sum(a * k, axis=1, keepdims=True) / kk)
        self.a = a
        # scale on a fixed 48^3 lattice
        g = [np.linspace(0, Ld, 48, endpoint=False) for Ld in self.lengths]
        Z, Y, X = np.meshgrid(g[2], g[1], g[0], indexing="ij")
        u = self.raw(X.ravel(), Y.ravel(), Z.ravel())
        mag = np.sqrt(np.max(np.sum(u * u, axis=0)))
        self.a *= self.amp / mag

    def kvec(self):
        L = np.asarray(self.lengths)
        return 2 * math.pi * self.m / L[None, :]

    def raw(self, x, y, z, chunk=65536):
        # exp(i k.x) = ex[mx] ey[my] ez[mz]: one complex exponential per axis and
        # integer wavenumber; the amplitudes on the dense (mx, my, mz) lattice
        # (zero off the ball) are contracted one axis at a time
        L = np.asarray(self.lengths)
        mi = self.m.astype(np.int64)
        lo = mi.min(axis=0)
        span = mi.max(axis=0) - lo + 1
        A = np.zeros((span[0], span[1], span[2], 3), complex)
        A[mi[:, 0] - lo[0], mi[:, 1] - lo[1], mi[:, 2] - lo[2]] = self.a
        A = A.reshape(span[0], -1)
        out = np.zeros((3, x.size))
        for s in range(0, x.size, chunk):
            cols = []
            for d, c in enumerate((x[s:s + chunk], y[s:s + chunk], z[s:s + chunk])):
                # powers of exp(i 2 pi c / L) from exp(i 2 pi lo c / L) on
                th = 2 * math.pi * c / L[d]
                pw = np.empty((c.size, span[d]), complex)
                pw[:, 0] = np.exp(1j * lo[d] * th)
                if span[d] > 1:
                    pw[:, 1:] = np.exp(1j * th)[:, None]
                cols.append(np.cumprod(pw, axis=1))
            t = (cols[0] @ A).reshape(-1, span[1], span[2], 3)
            t = np.einsum("pyzc,py->pzc", t, cols[1])
            out[:, s:s + chunk] = np.real(np.einsum("pzc,pz->cp", t, cols[2]))
        return out

    def __call__(self, x, y, z):
        return self.raw(np.ravel(x), np.ravel(y), np.ravel(z))


def perturbed_uniform_flow(x, y, z, modes, ma, gamma=GAMMA):
    """rho = 1, p = 1/(gamma Ma^2), u = (1,0,0) + u'(x)."""
    up = modes(x, y, z)
    pinf = 1.0 / (gamma * ma * ma)
    one = np.ones_like(x)
    return primitive_to_conservative(one, 1.0 + up[0], up[1], up[2], pinf * one, gamma)


def lamb_oseen_street(x, y, z, ma=0.2, gamma=GAMMA, a=1.0, b_over_a=0.281, yc=4.0,
                      core2=0.04, lx=8.0, noise=None):
    """Two staggered rows of Lamb-Oseen vortices u_theta = G/(2 pi r)(1-exp(-r^2/rc^2))
    (G = +1 upper row, -1 lower row, spacing a, row gap b), periodic images one
    period either side, on top of u = (1,0,0), rho = 1, p = 1/(gamma Ma^2)."""
    u = np.ones_like(x)
    v = np.zeros_like(x)
    b = b_over_a * a
    nv = int(round(lx / a))
    for row, (yy, G, xs) in enumerate(((yc + 0.5 * b, 1.0, 0.25 * a), (yc - 0.5 * b, -1.0, 0.75 * a))):
        for i in range(-nv, 2 * nv):
            cx = xs + i * a
            dx = x - cx
            dy = y - yy
            r2 = dx * dx + dy * dy + 1e-300
            # 1 - exp(-r^2/rc^2) is 1.0 in float64 beyond r^2 = 40 rc^2
            core = np.ones_like(r2)
            near = r2 < 40.0 * core2
            core[near] = 1.0 - np.exp(-r2[near] / core2)
            ut = (G / (2 * math.pi)) * core / r2  # u_theta / r
            u += -ut * dy
            v += ut * dx
    w = np.zeros_like(x)
    if noise is not None:
        up = noise(x, y, z)
        u += up[0]
        v += up[1]
        w += up[2]
    one = np.ones_like(x)
    return primitive_to_conservative(one, u, v, w, one / (gamma * ma * ma), gamma)


def sample(mesh, elem_p, fn):
    """U[5, n_sp]: ``fn(x, y, z) -> [5, npts]`` at every solution point."""
    X = solution_points(mesh, elem_p)
    return np.ascontiguousarray(fn(X[0], X[1], X[2]), dtype=np.float64)


# --------------------------------------------------------------------- configs
@dataclass
class Case:
    name: str
    mesh: dict
    elem_p: np.ndarray
    U: np.ndarray
    physics: int          # 0 Euler, 1 Navier-Stokes
    flux: int             # 0 Roe, 1 Rusanov
    gamma: float
    mu: float
    prandtl: float
    farfield: np.ndarray
    extra: dict

    @property
    def n_dof(self):
        return int(self.U.size)

    def desc(self):
        return dict(elem_xyz=self.mesh["elem_xyz"], elem_nbr=self.mesh["elem_nbr"],
                    elem_p=self.elem_p, physics=self.physics, flux=self.flux,
                    gamma=self.gamma, mu=self.mu, prandtl=self.prandtl,
                    farfield=self.farfield)


def _farfield(ma, gamma=GAMMA):
    return primitive_to_conservative(np.array(1.0), np.array(1.0), np.array(0.0),
                                     np.array(0.0), np.array(1.0 / (gamma * ma * ma)), gamma).astype(np.float64)


def case_vortex(nx=8, ny=8, nz=2, p=2, lengths=(10.0, 10.0, 2.5), center=(5.0, 5.0),
                ma=0.5, flux=1, elem_p=None, noise=0.0, seed=None):
    """Euler isentropic vortex on a periodic box (default: the 8x8x2, p = 2,
    Rusanov, Mach 0.5 case)."""
    mesh = box_mesh(nx, ny, nz, lengths, noise=noise, seed=seed)
    if elem_p is None:
        elem_p = np.full(mesh["n_elem"], p, dtype=np.int8)
    U = sample(mesh, elem_p, lambda x, y, z: vortex_field(x, y, z, center[0], center[1], ma=ma))
    return Case("vortex", mesh, np.asarray(elem_p, np.int8), U, 0, flux, GAMMA, 0.0, 0.72,
                _farfield(ma), dict(ma=ma, center=center, lengths=lengths))


def case_ns_mixed(nx=32, ny=32, nz=4, k=2, re=3900.0, ma=0.2, pvals=(1, 2, 3, 4),
                  pw=(0.4, 0.3, 0.2, 0.1), lengths=None, kmax_m=8, amp=0.1, noise_frac=0.05,
                  wall=False, flux=0):
    """Navier-Stokes, seeded mixed degree, perturbed vertices, divergence-free
    Fourier modes on a Mach ``ma`` base flow.  ``wall`` puts a no-slip adiabatic
    wall at y = 0 and far field at y = Ly (periodic in x and z)."""
    if lengths is None:
        h = 1.0 / nx
        lengths = (1.0, ny * h, nz * h)
    h = lengths[0] / nx
    periodic = (True, not wall, True)
    mesh = box_mesh(nx, ny, nz, lengths, periodic=periodic, noise=noise_frac * h,
                    seed=2000 + k, bc_lo=[BC_WALL] * 3, bc_hi=[BC_FARFIELD] * 3)
    elem_p = draw_p(mesh["n_elem"], pvals, pw, 1000 + k)
    modes = FourierModes(tuple(lengths), 2 * math.pi * kmax_m, amp, 3000 + k)
    U = sample(mesh, elem_p, lambda x, y, z: perturbed_uniform_flow(x, y, z, modes, ma))
    return Case("ns_mixed", mesh, elem_p, U, 1, flux, GAMMA, 1.0 / re, 0.72, _farfield(ma),
                dict(ma=ma, re=re, lengths=lengths))


def config(k, **over):
    """The five synthetic workloads (k = 1..5)."""
    if k == 1:
        return case_vortex(**over)
    if k == 2:
        return case_ns_mixed(32, 32, 4, k=2, **over)
    if k == 4:
        return case_ns_mixed(32, 32, 8, k=4, lengths=(1.0, 1.0, 0.25), wall=True, **over)
    if k == 5:
        return case_ns_mixed(128, 128, 8, k=5, re=60000.0, ma=0.1, pw=(0.3, 0.3, 0.25, 0.15),
                             lengths=(1.0, 1.0, 1.0 / 16), **over)
    if k == 3:
        return case_street(**over)
    raise ValueError(k)


def case_street(nx=64, ny=64, nz=8, elem_p=None, p_init=5, ma=0.2, re=3900.0):
    """Vortex-street field on [0,8]x[0,8]x[0,1]; the degree field is an input
    (the caller sets it, e.g. from the smoothness indicator)."""
    lengths = (8.0, 8.0, 1.0)
    mesh = box_mesh(nx, ny, nz, lengths)
    noise = FourierModes(lengths, 4 * 2 * math.pi / 8.0, 0.02, 3003)
    if elem_p is None:
        elem_p = np.full(mesh["n_elem"], p_init, dtype=np.int8)
    U = sample(mesh, elem_p, lambda x, y, z: lamb_oseen_street(x, y, z, ma=ma, noise=noise))
    return Case("street", mesh, np.asarray(elem_p, np.int8), U, 1, 0, GAMMA, 1.0 / re, 0.72,
                _farfield(ma), dict(ma=ma, re=re, lengths=lengths, noise=noise))


def resample(case, elem_p):
    """Same mesh and analytic field at a new degree field."""
    if case.name == "street":
        return case_street(*case.mesh["shape"], elem_p=elem_p, ma=case.extra["ma"], re=case.extra["re"])
    raise ValueError(case.name)


def random_direction(n_dof, seed, unit=True):
    v = np.random.default_rng(seed).normal(size=n_dof)
    if unit:
        v /= np.linalg.norm(v)
    return v
