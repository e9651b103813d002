"""Element-Jacobi preconditioner of section 2.3 and restarted GMRES with left
preconditioning (test infrastructure only): numpy, from the oracle's dense
Jacobian on small meshes.  Only the tests use it.

* Blocks: for every element, the diagonal block of sigma I - dR/dq, the rows
  and columns of the element's own DOF, ordered variable by variable and,
  inside a variable, as the element's solution points are stored.
* Apply: y_e = block_e^{-1} x_e for every element (numpy's dense solve).
* GMRES: Saad and Schultz's restarted GMRES with modified Gram-Schmidt on the
  left-preconditioned system P^{-1} A x = P^{-1} F from x = 0, stopping when
  the Arnoldi estimate of ||P^{-1} (F - A x)|| falls to tol ||P^{-1} F|| or the
  iteration budget is spent.
"""
from __future__ import annotations

import numpy as np


def element_dofs(sp_offset, n_sp):
    """Indices of every element's DOF in the state vector U[5][n_sp]
    (flattened), variable-major inside the element."""
    out = []
    for e in range(len(sp_offset) - 1):
        k = np.arange(sp_offset[e], sp_offset[e + 1])
        out.append(np.concatenate([v * n_sp + k for v in range(5)]))
    return out


def element_blocks(J, dofs, sigma):
    return [sigma * np.eye(len(ix)) - J[np.ix_(ix, ix)] for ix in dofs]


def apply(blocks, dofs, x):
    x = np.asarray(x, dtype=np.float64).ravel()
    y = np.empty_like(x)
    for B, ix in zip(blocks, dofs):
        y[ix] = np.linalg.solve(B, x[ix])
    return y


def gmres_left(matvec, precond, F, m, max_it, tol):
    """Returns (x, iterations, ||P^-1 r|| / ||P^-1 F|| estimate)."""
    F = np.asarray(F, dtype=np.float64).ravel()
    x = np.zeros_like(F)
    pF = precond(F)
    nF = np.linalg.norm(pF)
    if nF == 0.0:
        return x, 0, 0.0
    total = 0
    r = pF
    res = nF
    while True:
        beta = np.linalg.norm(r)
        V = [r / beta]
        H = np.zeros((m + 1, m))
        g = np.zeros(m + 1)
        g[0] = beta
        cs, sn = np.zeros(m), np.zeros(m)
        k = 0
        for j in range(m):
            w = precond(matvec(V[j]))
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            V.append(w / H[j + 1, j] if H[j + 1, j] > 0 else w)
            for i in range(j):
                a, b = H[i, j], H[i + 1, j]
                H[i, j], H[i + 1, j] = cs[i] * a + sn[i] * b, -sn[i] * a + cs[i] * b
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = (H[j, j] / den, H[j + 1, j] / den) if den > 0 else (1.0, 0.0)
            H[j, j], H[j + 1, j] = den, 0.0
            g[j + 1], g[j] = -sn[j] * g[j], cs[j] * g[j]
            res = abs(g[j + 1])
            total += 1
            k = j + 1
            if res <= tol * nF or total >= max_it:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + np.column_stack(V[:k]) @ y
        if res <= tol * nF or total >= max_it:
            break
        r = precond(F - matvec(x))
    return x, total, res / nF
