"""Pins of the oracle's nodal polynomial filter (CPU).

The filter (section 4.2) keeps the part of an element's polynomial that lies
in the degree p - 1 tensor space and scales the rest by 1 - alpha.  The pins
sample Legendre modes at the Gauss points (numpy's own Legendre basis), so a
wrong projection, a dropped direction or a wrong blend shows as a wrong
factor on some mode."""
import numpy as np
import pytest

from oracle import filter as F


def _grid(n):
    x = np.polynomial.legendre.leggauss(n)[0]
    z, y, xx = np.meshgrid(x, x, x, indexing="ij")  # [k][j][i], xi fastest
    return xx.reshape(-1), y.reshape(-1), z.reshape(-1)


def _mode(n, a, b, c):
    """P_a(xi) P_b(eta) P_c(zeta) at the n^3 Gauss points."""
    x, y, z = _grid(n)
    L = np.polynomial.legendre.Legendre.basis
    return L(a)(x) * L(b)(y) * L(c)(z)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_modes_below_the_top_are_kept(p):
    n = p + 1
    rng = np.random.default_rng(70 + p)
    u = np.zeros(n ** 3)
    for a in range(p):
        for b in range(p):
            for c in range(p):
                u += rng.normal() * _mode(n, a, b, c)
    np.testing.assert_allclose(F.filter_element(u, n, 0.2), u, rtol=0, atol=1e-13 * np.abs(u).max())


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("abc", ["x", "y", "z", "xy", "xyz"])
def test_a_top_mode_in_any_direction_is_scaled(p, abc):
    n = p + 1
    # the top mode in the named directions, a lower one (degree <= 1) in the others
    low = min(1, p - 1)
    a, b, c = (p if d in abc else low for d in "xyz")
    u = _mode(n, a, b, c)
    alpha = 0.2
    np.testing.assert_allclose(F.filter_element(u, n, alpha), (1 - alpha) * u, rtol=0, atol=1e-13)


def test_mixture_and_alpha_limits():
    p, n = 3, 4
    low = 0.7 * _mode(n, 2, 1, 0) - 1.3 * _mode(n, 0, 0, 2) + 2.0
    high = 0.9 * _mode(n, 3, 1, 0) + 0.4 * _mode(n, 1, 3, 2) - 0.5 * _mode(n, 3, 3, 3)
    u = low + high
    np.testing.assert_allclose(F.filter_element(u, n, 0.2), low + 0.8 * high, atol=1e-13)
    np.testing.assert_array_equal(F.filter_element(u, n, 0.0), u)
    full = F.filter_element(u, n, 1.0)
    np.testing.assert_allclose(full, low, atol=1e-13)
    # the projection is idempotent
    np.testing.assert_allclose(F.filter_element(full, n, 1.0), full, atol=1e-13)


def test_one_direction_against_a_least_squares_fit():
    """Data that varies along xi only: the filter along that line equals
    dropping the top coefficient of numpy's Legendre fit through the n points
    (a route that shares nothing with the oracle's Vandermonde inverse)."""
    rng = np.random.default_rng(5)
    for p in (2, 3, 4, 5):
        n = p + 1
        x1 = np.polynomial.legendre.leggauss(n)[0]
        f = np.exp(np.sin(3 * x1)) + rng.normal(size=n) * 0.1
        coef = np.polynomial.legendre.legfit(x1, f, p)
        trunc = np.polynomial.legendre.legval(x1, coef[:-1])
        want = 0.8 * f + 0.2 * trunc
        u = np.tile(f, n * n)  # same line for every (eta, zeta)
        got = F.filter_element(u, n, 0.2).reshape(n, n, n)
        for k in range(n):
            for j in range(n):
                np.testing.assert_allclose(got[k, j], want, atol=1e-13)


def test_elements_below_p_from_are_untouched():
    rng = np.random.default_rng(9)
    elem_p = np.array([1, 2, 3, 4, 5, 2, 3])
    U = rng.normal(size=(5, int(((elem_p + 1) ** 3).sum())))
    out = F.nodal_filter(elem_p, U, 0.2, 3)
    off = np.concatenate([[0], np.cumsum((elem_p + 1) ** 3)])
    for e, p in enumerate(elem_p):
        blk, ob = U[:, off[e]:off[e + 1]], out[:, off[e]:off[e + 1]]
        if p < 3:
            np.testing.assert_array_equal(ob, blk)
        else:
            assert np.abs(ob - blk).max() > 1e-3
            # the cell mean in reference space (mode 0) is kept
            w = np.polynomial.legendre.leggauss(p + 1)[1]
            W = np.einsum("k,j,i->kji", w, w, w).reshape(-1)
            np.testing.assert_allclose(ob @ W, blk @ W, rtol=1e-13)
