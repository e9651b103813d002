"""Degree selection of section 3.1 (test infrastructure only): the oracle's
statement of the refinement criteria and of the one-degree limit at faces,
in numpy.  Only the tests and the benchmark's reference leg use it; the
product path selects degrees on the device (fr_select_degrees).

* Criteria (section 3.1, the two threshold inequalities on the indicator):
  an element whose indicator exceeds nu_max times the largest indicator gets
  one degree more, one whose indicator is below nu_min times it one degree
  less; the result stays in [p_min, p_max].  Both inequalities are strict.
  "The largest indicator" (the paper's eta_{k,max}) is read two ways:
  scope "all", over every element, or scope "degree", over the elements of
  the same degree as the element.
* Limiter (section 3.1, neighbours differ by at most one degree): where a
  face joins degrees that differ by more than one, the lower side is raised
  (refinement wins) until no face does.  Boundary faces (negative neighbour
  ids) impose nothing.
"""
from __future__ import annotations

import numpy as np


def eta_maxima(p, eta, scope="all"):
    """The reference maximum of every element: the largest eta of all
    elements, or of the elements of the same degree."""
    p = np.asarray(p, dtype=np.int64)
    eta = np.asarray(eta, dtype=np.float64)
    if scope == "all":
        return np.full(len(p), eta.max() if len(eta) else 0.0)
    if scope != "degree":
        raise ValueError(scope)
    out = np.zeros(len(p))
    for k in np.unique(p):
        sel = p == k
        out[sel] = eta[sel].max()
    return out


def apply_criteria(p, eta, eta_max, nu_max=0.1, nu_min=0.001, p_min=1, p_max=5):
    """eta_max: a number, or one reference maximum per element."""
    p = np.asarray(p, dtype=np.int64)
    eta = np.asarray(eta, dtype=np.float64)
    up = eta > nu_max * eta_max
    down = eta < nu_min * eta_max
    return np.clip(p + up.astype(np.int64) - down.astype(np.int64), p_min, p_max)


def limit_jumps(p, elem_nbr, max_jump=1):
    """Raises the lower side of every face until no face joins degrees that
    differ by more than max_jump (a fixed point: one element at a time, in
    mesh order, repeated until nothing changes)."""
    p = np.asarray(p, dtype=np.int64).copy()
    nbr = np.asarray(elem_nbr)
    changed = True
    while changed:
        changed = False
        for e in range(len(p)):
            for nb in nbr[e]:
                if nb >= 0 and p[nb] - p[e] > max_jump:
                    p[e] = p[nb] - max_jump
                    changed = True
    return p


def select_degrees(p, eta, eta_max, elem_nbr, nu_max=0.1, nu_min=0.001, p_min=1, p_max=5, scope="all"):
    """Criteria, then the limiter: the degree field one adaptation chooses.
    With scope "all" eta_max is the global maximum (as returned with eta); with
    scope "degree" it is ignored and the per-degree maxima are used."""
    ref = eta_max if scope == "all" else eta_maxima(p, eta, "degree")
    return limit_jumps(apply_criteria(p, eta, ref, nu_max, nu_min, p_min, p_max), elem_nbr)


def indicator_degree_field(make_case, indicator, p_max=5, p_min=1, nu_max=0.1, nu_min=0.001, sweeps=4, scope="all"):
    """The degree field of an analytic workload: every element starts at p_max
    (the paper starts its adaptive runs at the highest degree); each sweep
    samples the field at the current degrees (``make_case(p)``), evaluates
    ``indicator(case) -> (eta, eta_max)`` and selects new degrees, until the
    field stops changing or ``sweeps`` sweeps are done."""
    case = make_case(None)
    p = np.full(case.mesh["n_elem"], p_max, np.int64)
    hist = []
    for _ in range(sweeps):
        case = make_case(p.astype(np.int8))
        eta, mx = indicator(case)
        pn = select_degrees(p, eta, mx, case.mesh["elem_nbr"], nu_max, nu_min, p_min, p_max, scope)
        hist.append(np.bincount(pn, minlength=p_max + 1)[1:].tolist())
        if np.array_equal(pn, p):
            break
        p = pn
    return p, hist
