"""Nodal polynomial filter (test infrastructure only, plain numpy).

Section 4.2 of the paper stabilises its under-resolved p^3 runs with the
nodal filter of Fischer and Mullen, applied to every element whose degree
exceeds two: the filtered solution is (1 - alpha) times the element's
solution plus alpha times its projection onto the degree p - 1 space
(p^2 for the paper's p^3 elements), with alpha = 0.2.  The projection is
taken as in the degree transfer of adaptation (oracle/projection.py: the
reference-space L2 projection onto the tensor space of degree p - 1), and
the projected polynomial is evaluated at the element's own solution points.
All five conservative variables are filtered.
"""
from __future__ import annotations

import numpy as np

from oracle.projection import project_element


def filter_element(u, n, alpha):
    """One variable of one element of size n = p + 1 (values at the n^3 Gauss
    points, xi fastest)."""
    low = project_element(u, n, n - 1)     # onto degree p - 1
    back = project_element(low, n - 1, n)  # that polynomial at the degree p points
    return (1.0 - alpha) * u + alpha * back


def nodal_filter(elem_p, U, alpha=0.2, p_from=3):
    """U [5, sum (p+1)^3] -> filtered copy; elements with p < p_from keep
    their values."""
    n = np.asarray(elem_p, dtype=np.int64) + 1
    off = np.concatenate([[0], np.cumsum(n ** 3)])
    out = np.array(U, dtype=np.float64, copy=True)
    for e in range(len(n)):
        if n[e] - 1 < p_from:
            continue
        for v in range(5):
            out[v, off[e]:off[e + 1]] = filter_element(U[v, off[e]:off[e + 1]], n[e], alpha)
    return out
