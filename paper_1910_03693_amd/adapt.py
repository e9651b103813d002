"""Degree selection from the spectral-decay indicator (section 3.1 of the
paper), host logic around the GPU indicator:

* criteria: raise p by one where eta > nu_max * eta_max, lower it by one where
  eta < nu_min * eta_max (nu_max = 0.1, nu_min = 0.001), p in [p_min, p_max];
* limiter: the degree difference across a face is at most one; where it is
  larger the lower side is raised (refinement wins), iterated to a fixed
  point.

``indicator_degree_field`` starts every element at p_max (the paper starts its
adaptive runs at the highest degree), samples the analytic field at the
current degrees, evaluates the indicator of rho u on the GPU and applies the
criteria until the field stops changing (at most ``sweeps`` times), then
applies the limiter.
"""
from __future__ import annotations

import numpy as np


def apply_criteria(p, eta, eta_max, nu_max=0.1, nu_min=0.001, p_min=1, p_max=5):
    p = np.asarray(p, dtype=np.int64)
    up = eta > nu_max * eta_max
    down = eta < nu_min * eta_max
    return np.clip(p + up.astype(np.int64) - down.astype(np.int64), p_min, p_max).astype(np.int8)


def limit_jumps(p, elem_nbr, max_jump=1):
    p = np.asarray(p, dtype=np.int64).copy()
    nbr = np.asarray(elem_nbr)
    while True:
        pn = np.where(nbr >= 0, p[np.clip(nbr, 0, None)], -10)
        need = np.maximum(p, pn.max(axis=1) - max_jump)
        if np.array_equal(need, p):
            return p.astype(np.int8)
        p = need


def indicator_degree_field(make_case, p_max=5, p_min=1, nu_max=0.1, nu_min=0.001, sweeps=4, var=1):
    """``make_case(elem_p)`` builds the workload at a degree field; returns the
    final degree field and the per-sweep histograms."""
    import torch

    from . import frx

    case = make_case(None)
    p = np.full(case.mesh["n_elem"], p_max, np.int8)
    hist = []
    for _ in range(sweeps):
        case = make_case(p)
        ctx = frx.Context.from_case(case)
        U = torch.tensor(case.U, device="cuda")
        eta, mx = ctx.indicator(U, var=var)
        pn = apply_criteria(p, eta.cpu().numpy(), float(mx.item()), nu_max, nu_min, p_min, p_max)
        ctx.close()
        hist.append(np.bincount(pn, minlength=p_max + 1)[1:].tolist())
        if np.array_equal(pn, p):
            break
        p = pn
    p = limit_jumps(p, case.mesh["elem_nbr"])
    return p, hist


def adapt_step(case, ctx, U, nu_max=0.1, nu_min=0.001, p_min=1, p_max=5, var=1):
    """One p-adaptation on the device: degrees from the indicator, criteria and
    face limiter (fr_select_degrees), a context for the new degree field (new
    degree buckets and face lists), the state projected onto it (fr_project).
    Returns (new case description, new context, new state)."""
    import dataclasses

    from . import frx

    p_new = ctx.select_degrees(U, var, nu_max, nu_min, p_min, p_max).cpu().numpy()
    new_case = dataclasses.replace(case, elem_p=p_new.astype(np.int8), U=None)
    new_ctx = frx.Context.from_case(new_case)
    return new_case, new_ctx, ctx.project_to(U, new_ctx)
