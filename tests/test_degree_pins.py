"""Pins of the oracle's degree selection (section 3.1: the two threshold
criteria on the spectral-decay indicator and the one-degree limit at faces),
on hand-made inputs whose answers are worked out by hand."""
import numpy as np

from oracle import degrees as D
from paper_1910_03693_amd import inputs as I


def test_criteria_raise_lower_and_clamp():
    p = np.array([1, 2, 3, 5, 1, 3], np.int8)
    eta = np.array([0.5, 0.05, 1e-5, 0.9, 1e-6, 0.01])
    # eta_max = 1: raise above 0.1, lower below 0.001; clamp to [1, 5]
    assert D.apply_criteria(p, eta, 1.0).tolist() == [2, 2, 2, 5, 1, 3]


def test_criteria_thresholds_are_strict_and_scale_with_eta_max():
    p = np.array([3, 3, 3, 3], np.int8)
    # exactly at nu_max * eta_max and nu_min * eta_max: no change either way
    eta = np.array([0.2, 0.002, 0.2 + 1e-12, 0.002 - 1e-12])
    assert D.apply_criteria(p, eta, 2.0).tolist() == [3, 3, 4, 2]
    # other thresholds and bounds
    out = D.apply_criteria(np.array([2, 4, 3]), np.array([0.6, 0.6, 0.0]), 1.0, nu_max=0.5, nu_min=0.1,
                           p_min=2, p_max=4)
    assert out.tolist() == [3, 4, 2]


def test_limiter_raises_lower_side_to_fixed_point():
    m = I.box_mesh(5, 1, 1, (5.0, 1.0, 1.0), periodic=(False, True, True))
    p = np.array([5, 1, 1, 1, 1], np.int8)
    assert D.limit_jumps(p, m["elem_nbr"]).tolist() == [5, 4, 3, 2, 1]
    # already admissible fields are unchanged
    q = np.array([1, 2, 3, 2, 1], np.int8)
    assert D.limit_jumps(q, m["elem_nbr"]).tolist() == q.tolist()
    # periodic in x: the chain wraps round the last face
    mp = I.box_mesh(5, 1, 1, (5.0, 1.0, 1.0))
    assert D.limit_jumps(np.array([5, 1, 1, 1, 1]), mp["elem_nbr"]).tolist() == [5, 4, 3, 3, 4]


def test_limiter_is_the_least_admissible_field_above():
    """Brute force on a small periodic mesh: the limited field is admissible,
    never below the input, and every admissible field above the input is
    above it (the least fixed point, whatever the sweep order)."""
    rng = np.random.default_rng(0)
    m = I.box_mesh(4, 4, 2, (1.0, 1.0, 0.5))
    nb = m["elem_nbr"]
    for trial in range(5):
        r = rng.integers(1, 6, m["n_elem"])
        lim = D.limit_jumps(r, nb)
        assert np.all(lim >= r)
        assert np.all(np.abs(lim[:, None] - lim[nb]) <= 1)
        # any admissible field above r: raise random elements of lim, then limit
        up = D.limit_jumps(np.maximum(r, lim - rng.integers(0, 2, m["n_elem"])), nb)
        assert np.all(up >= lim)
        # lowering any single raised element breaks admissibility or the bound
        raised = np.nonzero(lim > r)[0]
        for e in raised[:10]:
            low = lim.copy()
            low[e] -= 1
            assert np.any(np.abs(low[:, None] - low[nb]) > 1)


def test_limiter_ignores_boundary_faces():
    m = I.box_mesh(3, 1, 1, (3.0, 1.0, 1.0), periodic=(False, True, True))
    nb = np.array(m["elem_nbr"])
    assert (nb < 0).any()
    assert D.limit_jumps(np.array([1, 3, 1]), nb).tolist() == [2, 3, 2]


def test_selection_is_criteria_then_limiter():
    m = I.box_mesh(4, 1, 1, (4.0, 1.0, 1.0), periodic=(False, True, True))
    p = np.array([4, 2, 2, 2])
    eta = np.array([1.0, 1e-6, 1e-6, 0.05])
    # criteria: [5, 1, 1, 2]; limiter: [5, 4, 3, 2]
    assert D.select_degrees(p, eta, 1.0, m["elem_nbr"]).tolist() == [5, 4, 3, 2]


def test_same_degree_maxima():
    p = np.array([1, 1, 2, 2, 3])
    eta = np.array([0.5, 1e-4, 0.01, 1e-7, 2e-3])
    assert D.eta_maxima(p, eta, "all").tolist() == [0.5] * 5
    assert D.eta_maxima(p, eta, "degree").tolist() == [0.5, 0.5, 0.01, 0.01, 2e-3]
    # criteria against each reference, worked out by hand
    assert D.apply_criteria(p, eta, D.eta_maxima(p, eta, "all")).tolist() == [2, 1, 2, 1, 3]
    assert D.apply_criteria(p, eta, D.eta_maxima(p, eta, "degree")).tolist() == [2, 1, 3, 1, 4]
    # through select_degrees, on elements that share no face
    nbr = -np.ones((5, 6), dtype=np.int32)
    assert D.select_degrees(p, eta, 0.5, nbr, scope="degree").tolist() == [2, 1, 3, 1, 4]
    assert D.select_degrees(p, eta, 0.5, nbr, scope="all").tolist() == [2, 1, 2, 1, 3]
