"""Pins of the oracle's element-Jacobi preconditioner and left-preconditioned
GMRES (section 2.3) on small meshes, against dense linear algebra and finite
differences."""
import numpy as np
import pytest

from oracle import precond as PC
from paper_1910_03693_amd import inputs as I


def _small(oracle_mod, nx=3, ny=2, nz=2, pvals=(1, 2), k=81):
    c = I.case_ns_mixed(nx, ny, nz, k=k, lengths=(1.0, 0.7, 0.6), pvals=pvals, pw=(1,) * len(pvals), re=200.0, ma=0.3)
    orc = oracle_mod.Oracle.from_case(c)
    off = I.sp_offsets(c.elem_p)
    return c, orc, PC.element_dofs(off, orc.n_sp)


def test_blocks_are_the_element_jacobians_by_finite_differences(oracle_mod):
    # each block, minus sigma I, is -dR_e/dU_e: central differences of the
    # residual in the element's own DOF, read in its own rows
    c, orc, dofs = _small(oracle_mod)
    J = orc.jacobian(c.U)
    sigma = 40.0
    blocks = PC.element_blocks(J, dofs, sigma)
    U = c.U.ravel()
    e = 3
    ix = dofs[e]
    h = 1e-6
    for j in range(0, len(ix), 7):
        up, um = U.copy(), U.copy()
        up[ix[j]] += h
        um[ix[j]] -= h
        col = (orc.residual(up.reshape(c.U.shape)).ravel() - orc.residual(um.reshape(c.U.shape)).ravel()) / (2 * h)
        expect = sigma * (np.arange(len(ix)) == j) - col[ix]
        assert np.max(np.abs(blocks[e][:, j] - expect)) <= 1e-6 * np.max(np.abs(expect))


def test_single_element_block_is_the_whole_matrix_one_iteration(oracle_mod):
    # one self-periodic element: P = A, so P^-1 A = I and GMRES needs one step
    c, orc, dofs = _small(oracle_mod, 1, 1, 1, pvals=(2,))
    J = orc.jacobian(c.U)
    sigma = 30.0
    A = sigma * np.eye(J.shape[0]) - J
    blocks = PC.element_blocks(J, dofs, sigma)
    F = np.random.default_rng(5).normal(size=J.shape[0])
    x, its, rr = PC.gmres_left(lambda v: A @ v, lambda v: PC.apply(blocks, dofs, v), F, 10, 10, 1e-12)
    assert its == 1
    assert np.linalg.norm(x - np.linalg.solve(A, F)) <= 1e-10 * np.linalg.norm(x)


def test_preconditioned_gmres_full_space_is_the_dense_solve(oracle_mod):
    c, orc, dofs = _small(oracle_mod)
    J = orc.jacobian(c.U)
    sigma = 25.0
    A = sigma * np.eye(J.shape[0]) - J
    blocks = PC.element_blocks(J, dofs, sigma)
    P = lambda v: PC.apply(blocks, dofs, v)
    F = np.random.default_rng(6).normal(size=J.shape[0])
    x, its, rr = PC.gmres_left(lambda v: A @ v, P, F, J.shape[0], J.shape[0], 1e-13)
    xd = np.linalg.solve(A, F)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
    # restarted: the stop test holds for the preconditioned residual, and the
    # preconditioned system needs fewer products than the plain one
    x2, its2, rr2 = PC.gmres_left(lambda v: A @ v, P, F, 8, 400, 1e-8)
    assert np.linalg.norm(P(F - A @ x2)) <= 1.01e-8 * np.linalg.norm(P(F))
    x3, its3, rr3 = PC.gmres_left(lambda v: A @ v, lambda v: v, F, 8, 400, 1e-8)
    assert its2 < its3
