"""Host logic of the degree selection (section 3.1 criteria and the
one-degree limit at faces), on hand-made inputs."""
import numpy as np

from paper_1910_03693_amd import adapt
from paper_1910_03693_amd import inputs as I


def test_criteria_raise_lower_and_clamp():
    p = np.array([1, 2, 3, 5, 1, 3], np.int8)
    eta = np.array([0.5, 0.05, 1e-5, 0.9, 1e-6, 0.01])
    # eta_max = 1: raise above 0.1, lower below 0.001
    out = adapt.apply_criteria(p, eta, 1.0)
    assert out.tolist() == [2, 2, 2, 5, 1, 3]


def test_limiter_raises_lower_side_to_fixed_point():
    m = I.box_mesh(5, 1, 1, (5.0, 1.0, 1.0), periodic=(False, True, True))
    p = np.array([5, 1, 1, 1, 1], np.int8)
    out = adapt.limit_jumps(p, m["elem_nbr"])
    assert out.tolist() == [5, 4, 3, 2, 1]
    # already admissible fields are unchanged; the result never lowers a degree
    q = np.array([1, 2, 3, 2, 1], np.int8)
    assert adapt.limit_jumps(q, m["elem_nbr"]).tolist() == q.tolist()
    rng = np.random.default_rng(0)
    m3 = I.box_mesh(4, 4, 2, (1.0, 1.0, 0.5))
    r = rng.integers(1, 6, m3["n_elem"]).astype(np.int8)
    lim = adapt.limit_jumps(r, m3["elem_nbr"])
    assert np.all(lim >= r)
    nb = m3["elem_nbr"]
    assert np.all(np.abs(lim[:, None].astype(int) - lim[nb].astype(int)) <= 1)
