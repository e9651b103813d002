"""Projection of a solution between two degree fields on the same mesh (test
infrastructure only, plain numpy).

Section 3.1 of the paper changes an element's degree by one after each time
step and obtains the lower-degree solution by projecting from the degree p
space to the degree p - 1 space; the transfer itself is not spelled out.
Reading taken here, element by element in reference coordinates:

* to a lower degree: the L2 projection onto the tensor space Q_{p'} (with
  p' < p), i.e. the Legendre expansion of the element's polynomial truncated to
  modes of index <= p' in every direction (the same projection the spectral-
  decay indicator uses);
* to an equal or higher degree: the element's polynomial evaluated at the new
  solution points (exact).

The element's polynomial is its tensor Lagrange interpolant through the
Gauss-Legendre solution points; its Legendre coefficients come from solving
the Vandermonde system V c = u (V_ik = P_k(x_i)) direction by direction.
"""
from __future__ import annotations

import numpy as np


def _nodes(n):
    x, _ = np.polynomial.legendre.leggauss(n)
    return x


def _vandermonde(x, nmodes):
    # V[i, k] = P_k(x_i)
    return np.stack([np.polynomial.legendre.Legendre.basis(k)(x) for k in range(nmodes)], axis=1)


def modal_coefficients(u, n):
    """Legendre coefficients c[a, b, c] of the element polynomial through the
    values u[k][j][i] (i along xi fastest) at n^3 Gauss points."""
    V = _vandermonde(_nodes(n), n)
    Vi = np.linalg.inv(V)
    c = u.reshape(n, n, n)  # [z][y][x]
    c = np.einsum("ai,zyi->zya", Vi, c)
    c = np.einsum("bj,zjx->zbx", Vi, c)
    c = np.einsum("ck,kyx->cyx", Vi, c)
    return c  # [mode_z][mode_y][mode_x]


def evaluate_modes(c, n):
    """Values at the n^3 Gauss points of the Legendre series c (any size <= n
    per direction; missing modes are zero)."""
    m = c.shape[0]
    V = _vandermonde(_nodes(n), m)
    u = np.einsum("ia,zya->zyi", V, c)
    u = np.einsum("jb,zbx->zjx", V, u)
    u = np.einsum("kc,cyx->kyx", V, u)
    return u.reshape(-1)


def project_element(u, n_src, n_dst):
    c = modal_coefficients(u, n_src)
    m = min(n_src, n_dst)
    return evaluate_modes(c[:m, :m, :m], n_dst)


def project(elem_p_src, U_src, elem_p_dst):
    """U_src [5, sum (p_src+1)^3] -> U_dst [5, sum (p_dst+1)^3], element by
    element in mesh order."""
    ps = np.asarray(elem_p_src, dtype=np.int64) + 1
    pd = np.asarray(elem_p_dst, dtype=np.int64) + 1
    os_ = np.concatenate([[0], np.cumsum(ps ** 3)])
    od = np.concatenate([[0], np.cumsum(pd ** 3)])
    out = np.zeros((5, od[-1]))
    for e in range(len(ps)):
        for v in range(5):
            out[v, od[e]:od[e + 1]] = project_element(U_src[v, os_[e]:os_[e + 1]], ps[e], pd[e])
    return out
