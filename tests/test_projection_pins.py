"""Pins of the oracle's projection between degree fields (CPU)."""
import numpy as np
import pytest

from oracle import projection as P


def _poly(x, y, z, deg, rng):
    # separable-sum polynomial of degree <= deg in each direction
    a = rng.normal(size=(deg + 1, deg + 1, deg + 1))
    out = np.zeros_like(x)
    for i in range(deg + 1):
        for j in range(deg + 1):
            for k in range(deg + 1):
                out += a[k, j, i] * x ** i * y ** j * z ** k
    return out


def _points(n):
    x = np.polynomial.legendre.leggauss(n)[0]
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return X.reshape(-1), Y.reshape(-1), Z.reshape(-1)


@pytest.mark.parametrize("ns,nd", [(2, 3), (3, 2), (4, 6), (6, 4), (5, 5), (3, 6), (6, 2)])
def test_polynomials_of_the_common_degree_are_reproduced(ns, nd):
    rng = np.random.default_rng(ns * 10 + nd)
    deg = min(ns, nd) - 1
    xs = _points(ns)
    xd = _points(nd)
    u = _poly(*xs, deg, rng)
    rng = np.random.default_rng(ns * 10 + nd)
    ref = _poly(*xd, deg, rng)
    got = P.project_element(u, ns, nd)
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("ns,nd", [(3, 2), (5, 3), (6, 5), (4, 2)])
def test_lowering_is_l2_orthogonal(ns, nd):
    """u - Pu is orthogonal to every Q_{nd-1} polynomial under the ns-point
    Gauss rule (exact for these products)."""
    rng = np.random.default_rng(7)
    u = rng.normal(size=ns ** 3)
    pu_at_src = P.project_element(P.project_element(u, ns, nd), nd, ns)  # Pu evaluated at the source points
    r = u - pu_at_src
    x, w = np.polynomial.legendre.leggauss(ns)
    W = (w[:, None, None] * w[None, :, None] * w[None, None, :]).reshape(-1)
    X, Y, Z = _points(ns)
    for i in range(nd):
        for j in range(nd):
            for k in range(nd):
                phi = X ** i * Y ** j * Z ** k
                assert abs(np.sum(W * r * phi)) <= 1e-12 * np.sqrt(np.sum(W * u * u))


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_raise_then_lower_is_identity(n):
    rng = np.random.default_rng(n)
    u = rng.normal(size=n ** 3)
    back = P.project_element(P.project_element(u, n, n + 1), n + 1, n)
    assert np.allclose(back, u, rtol=0, atol=1e-12 * np.abs(u).max())


def test_reference_mean_is_kept():
    rng = np.random.default_rng(3)
    for ns, nd in [(5, 2), (4, 1 + 1), (3, 6)]:
        u = rng.normal(size=ns ** 3)
        x, w = np.polynomial.legendre.leggauss(ns)
        W = (w[:, None, None] * w[None, :, None] * w[None, None, :]).reshape(-1)
        xd, wd = np.polynomial.legendre.leggauss(nd)
        Wd = (wd[:, None, None] * wd[None, :, None] * wd[None, None, :]).reshape(-1)
        assert abs(np.sum(W * u) - np.sum(Wd * P.project_element(u, ns, nd))) <= 1e-12 * np.abs(u).sum()


def test_whole_field_projection_layout():
    rng = np.random.default_rng(11)
    ps = np.array([1, 4, 2, 5, 3], np.int8)
    pd = np.array([2, 3, 2, 4, 4], np.int8)
    U = rng.normal(size=(5, int(((ps.astype(int) + 1) ** 3).sum())))
    out = P.project(ps, U, pd)
    assert out.shape == (5, int(((pd.astype(int) + 1) ** 3).sum()))
    # element 2 keeps its degree: unchanged
    o_s = np.concatenate([[0], np.cumsum((ps.astype(int) + 1) ** 3)])
    o_d = np.concatenate([[0], np.cumsum((pd.astype(int) + 1) ** 3)])
    assert np.allclose(out[:, o_d[2]:o_d[3]], U[:, o_s[2]:o_s[3]], rtol=0, atol=1e-13)
