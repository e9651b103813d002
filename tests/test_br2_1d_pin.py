"""Pin of the oracle's viscous (BR2) and inviscid face terms against a
one-dimensional FR scheme written here from the method's definitions.

On a uniform Cartesian box that is periodic in every direction, with one
element across two of the axes, a state that varies along the third axis
only and has no transverse velocity turns the three-dimensional FR operator
into the one-dimensional FR discretisation of the 1-D Navier-Stokes
equations for mass, the axial momentum and energy (section 2.2: tensor Gauss
points, DG correction functions, common solution and BR2 common gradient of
eq. com_q / com_grad_q, Roe or Rusanov common flux of eq. invis_com; the
readings of the paper that the oracle takes: BR2 gradient traces are the
face values of the uncorrected physical gradient, the liftings are
r = (2/h) g'(face) (q_com - q) with penalty 1, the interior gradient is the
corrected one, the common solution is the average of the conservative
states).  The reference below is plain numpy on the 1-D chain of elements,
with its own Legendre-based operators; it shares no code with the oracle.

The transverse momentum is not zero in the three-dimensional scheme: on the
faces across the axis the stress -(2/3) mu div(u) of the common flux takes
the uncorrected gradient trace, the local flux the corrected gradient, and
their difference enters through both correction functions of the element
(its two faces there are the same periodic face).  That term is predicted in
closed form and checked as well, which pins the bulk-viscosity part of the
Stokes stress.
"""
import numpy as np
import pytest
from numpy.polynomial import legendre as Lg

from paper_1910_03693_amd import inputs as I

GAMMA = 1.4
PR = 0.72


# ------------------------------------------------------------- 1-D operators
def ops(p):
    """Gauss points, derivative matrix, endpoint rows and DG correction slopes
    of degree p, from Legendre polynomials (numpy's basis)."""
    n = p + 1
    x, w = Lg.leggauss(n)
    V = Lg.legvander(x, p)                       # V[i, j] = P_j(x_i)
    Vi = np.linalg.inv(V)                        # Lagrange basis in Legendre coefficients
    Vd = np.stack([Lg.legval(x, Lg.legder(np.eye(n)[j])) for j in range(n)], axis=1)
    D = Vd @ Vi                                  # D[i, m] = l_m'(x_i)
    lm = Lg.legvander(np.array([-1.0]), p)[0] @ Vi
    lp = Lg.legvander(np.array([1.0]), p)[0] @ Vi
    # right Radau g_R = (P_p + P_{p+1}) / 2 (g_R(1) = 1, g_R(-1) = 0) and g_L(x) = g_R(-x)
    cR = np.zeros(p + 2)
    cR[p] = cR[p + 1] = 0.5
    cL = np.zeros(p + 2)
    cL[p] = 0.5 * (-1) ** p
    cL[p + 1] = -0.5 * (-1) ** p
    gRp = Lg.legval(x, Lg.legder(cR))
    gLp = Lg.legval(x, Lg.legder(cL))
    gR1 = Lg.legval(1.0, Lg.legder(cR))          # g_R'(+1)
    gLm1 = Lg.legval(-1.0, Lg.legder(cL))        # g_L'(-1)
    return dict(x=x, w=w, D=D, lm=lm, lp=lp, gLp=gLp, gRp=gRp, gR1=gR1, gLm1=gLm1)


# ------------------------------------------------------ 1-D physics (rho, m, E)
def pressure(q):
    return (GAMMA - 1.0) * (q[..., 2] - 0.5 * q[..., 1] ** 2 / q[..., 0])


def f_inv(q):
    u = q[..., 1] / q[..., 0]
    p = pressure(q)
    return np.stack([q[..., 1], q[..., 1] * u + p, (q[..., 2] + p) * u], axis=-1)


def visc_parts(q, g, mu):
    """u_x, T_x (chain rule from the conservative gradient g) and the 1-D
    viscous flux (0, tau_xx, u tau_xx + kappa T_x), tau_xx = 4/3 mu u_x."""
    rho, m, E = q[..., 0], q[..., 1], q[..., 2]
    u = m / rho
    ux = (g[..., 1] - u * g[..., 0]) / rho
    e = E / rho
    ex = (g[..., 2] - e * g[..., 0]) / rho
    Tx = (GAMMA - 1.0) * (ex - u * ux)
    kappa = mu * GAMMA / ((GAMMA - 1.0) * PR)
    tau = 4.0 / 3.0 * mu * ux
    fv = np.stack([np.zeros_like(tau), tau, u * tau + kappa * Tx], axis=-1)
    return ux, fv


def roe(qL, qR):
    rL, rR = qL[0], qR[0]
    uL, uR = qL[1] / rL, qR[1] / rR
    pL, pR = pressure(qL), pressure(qR)
    HL, HR = (qL[2] + pL) / rL, (qR[2] + pR) / rR
    sL, sR = np.sqrt(rL), np.sqrt(rR)
    u = (sL * uL + sR * uR) / (sL + sR)
    H = (sL * HL + sR * HR) / (sL + sR)
    c = np.sqrt((GAMMA - 1.0) * (H - 0.5 * u * u))
    rho = sL * sR
    dp, du, dr = pR - pL, uR - uL, rR - rL
    a1 = (dp - rho * c * du) / (2 * c * c)
    a2 = dr - dp / (c * c)
    a3 = (dp + rho * c * du) / (2 * c * c)
    r1 = np.array([1.0, u - c, H - u * c])
    r2 = np.array([1.0, u, 0.5 * u * u])
    r3 = np.array([1.0, u + c, H + u * c])
    diss = abs(u - c) * a1 * r1 + abs(u) * a2 * r2 + abs(u + c) * a3 * r3
    return 0.5 * (f_inv(qL) + f_inv(qR)) - 0.5 * diss


def rusanov(qL, qR):
    cL = np.sqrt(GAMMA * pressure(qL) / qL[0])
    cR = np.sqrt(GAMMA * pressure(qR) / qR[0])
    lam = max(abs(qL[1] / qL[0]) + cL, abs(qR[1] / qR[0]) + cR)
    return 0.5 * (f_inv(qL) + f_inv(qR)) - 0.5 * lam * (qR - qL)


def fr_1d(qs, degs, h, mu, flux):
    """Residual dq/dt of the periodic 1-D chain: qs[k] is [n_k, 3] at the Gauss
    points of element k (degree degs[k], width h).  Also returns, per element,
    u_x from the uncorrected and from the corrected gradient at its points."""
    K = len(qs)
    O = [ops(p) for p in degs]
    qm = [O[k]["lm"] @ qs[k] for k in range(K)]          # left traces
    qp = [O[k]["lp"] @ qs[k] for k in range(K)]          # right traces
    gu = [2.0 / h * (O[k]["D"] @ qs[k]) for k in range(K)]  # uncorrected gradient
    # interface k+1/2 between element k (left) and k+1 (right)
    qc = [0.5 * (qp[k] + qm[(k + 1) % K]) for k in range(K)]
    gc = []
    for k in range(K):
        r = (k + 1) % K
        gl = O[k]["lp"] @ gu[k]                          # uncorrected gradient traces
        gr = O[r]["lm"] @ gu[r]
        rl = 2.0 / h * O[k]["gR1"] * (qc[k] - qp[k])      # liftings of the two jumps
        rr = 2.0 / h * O[r]["gLm1"] * (qc[k] - qm[r])
        gc.append(0.5 * (gl + rl + gr + rr))
    R, ux_unc, ux_cor = [], [], []
    for k in range(K):
        o = O[k]
        cl, cr = qc[(k - 1) % K], qc[k]
        g = 2.0 / h * (o["D"] @ qs[k] + np.outer(o["gLp"], cl - qm[k]) + np.outer(o["gRp"], cr - qp[k]))
        f = f_inv(qs[k])
        if mu > 0.0:
            uxc, fv = visc_parts(qs[k], g, mu)
            uxu, _ = visc_parts(qs[k], gu[k], mu)
            f = f - fv
            ux_unc.append(uxu)
            ux_cor.append(uxc)
        fm, fp = o["lm"] @ f, o["lp"] @ f
        fcom = []
        for j in ((k - 1) % K, k):
            a, b = j, (j + 1) % K
            fs = flux(qp[a], qm[b])
            if mu > 0.0:
                _, fvc = visc_parts(qc[j], gc[j], mu)
                fs = fs - fvc
            fcom.append(fs)
        R.append(-2.0 / h * (o["D"] @ f + np.outer(o["gLp"], fcom[0] - fm) + np.outer(o["gRp"], fcom[1] - fp)))
    return R, ux_unc, ux_cor


# --------------------------------------------------------------- the pin
def _state(s, L):
    """(rho, m, E) of a smooth periodic 1-D state at coordinate s."""
    k = 2.0 * np.pi / L
    rho = 1.0 + 0.2 * np.sin(k * s) + 0.05 * np.cos(3 * k * s)
    u = 0.4 + 0.3 * np.cos(k * s + 0.3)
    p = 1.0 / (GAMMA * 0.5 ** 2) * (1.0 + 0.1 * np.sin(2 * k * s + 0.7))
    return np.stack([rho, rho * u, p / (GAMMA - 1.0) + 0.5 * rho * u * u], axis=-1)


CASES = [
    ("euler_roe_uniform", 0.0, 0, [3, 3, 3, 3]),
    ("euler_rusanov_mixed", 0.0, 1, [1, 3, 2, 4, 2]),
    ("ns_roe_uniform", 0.05, 0, [2, 2, 2, 2, 2]),
    ("ns_roe_mixed", 0.05, 0, [1, 3, 2, 4, 2]),
    ("ns_rusanov_mixed", 0.02, 1, [4, 1, 3, 2]),
]


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("name,mu,flux,degs", CASES, ids=[c[0] for c in CASES])
def test_oracle_reduces_to_1d_fr_br2(oracle_mod, axis, name, mu, flux, degs):
    K = len(degs)
    L = 2.0 * K * 0.75
    h = L / K
    shape = [1, 1, 1]
    shape[axis] = K
    lengths = [0.9, 1.3, 0.7]
    lengths[axis] = L
    mesh = I.box_mesh(*shape, lengths)
    elem_p = np.asarray(degs, dtype=np.int8)
    X = I.solution_points(mesh, elem_p)
    q1 = _state(X[axis], L)                       # [n_sp, 3]
    U = np.zeros((5, X.shape[1]))
    U[0], U[1 + axis], U[4] = q1[:, 0], q1[:, 1], q1[:, 2]
    orc = oracle_mod.Oracle(mesh["elem_xyz"], mesh["elem_nbr"], elem_p, 1 if mu > 0 else 0, flux, GAMMA, mu, PR)
    R3 = orc.residual(U)

    # the 1-D chain at the Gauss points of each element
    off = I.sp_offsets(elem_p)
    qs = []
    for k, p in enumerate(degs):
        x = ops(p)["x"]
        qs.append(_state(mesh["elem_xyz"][k, 0, axis] + (x + 1.0) * h / 2.0, L))
    R1, ux_unc, ux_cor = fr_1d(qs, degs, h, mu, roe if flux == 0 else rusanov)

    scale = max(np.max(np.abs(r)) for r in R1)
    worst = 0.0
    for k, p in enumerate(degs):
        n = p + 1
        idx = np.arange(n ** 3)
        i = [idx % n, (idx // n) % n, idx // (n * n)]   # (xi, eta, zeta) indices, xi fastest
        seg = slice(off[k], off[k + 1])
        for v3, v1 in ((0, 0), (1 + axis, 1), (4, 2)):
            worst = max(worst, np.max(np.abs(R3[v3, seg] - R1[k][i[axis], v1])))
        o = ops(p)
        for b in range(3):
            if b == axis:
                continue
            if mu > 0.0:
                # both faces across axis b are the one periodic face of the element:
                # f_com - f_loc = (2/3) mu (u_x uncorrected - u_x corrected)
                hb = lengths[b]
                delta = 2.0 / 3.0 * mu * (ux_unc[k] - ux_cor[k])
                pred = -2.0 / hb * (o["gLp"][i[b]] + o["gRp"][i[b]]) * delta[i[axis]]
            else:
                pred = np.zeros(n ** 3)
            worst = max(worst, np.max(np.abs(R3[1 + b, seg] - pred)))
    assert worst <= 1e-11 * scale, (name, axis, worst, scale)
