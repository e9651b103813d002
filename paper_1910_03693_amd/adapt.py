"""p-adaptation driver (section 3.1 of the paper) around the device calls.

``indicator_degree_field`` builds the degree field of an analytic workload:
every element starts at p_max (the paper starts its adaptive runs at the
highest degree); each sweep samples the field at the current degrees and lets
the device choose new ones with fr_select_degrees (indicator of rho u,
criteria nu_max = 0.1 / nu_min = 0.001, one-degree face limiter), until the
field stops changing (at most ``sweeps`` sweeps).

``adapt_step`` is one adaptation of a running solution: degrees from
fr_select_degrees, a context for the new degree field, the state moved onto
it by fr_project.
"""
from __future__ import annotations

import numpy as np


def indicator_degree_field(make_case, p_max=5, p_min=1, nu_max=0.1, nu_min=0.001, sweeps=4, var=1, eta_max_scope=0):
    """``make_case(elem_p)`` builds the workload at a degree field; returns the
    final degree field and the per-sweep histograms."""
    import torch

    from . import frx

    case = make_case(None)
    p = np.full(case.mesh["n_elem"], p_max, np.int8)
    hist = []
    for _ in range(sweeps):
        case = make_case(p)
        ctx = frx.Context.from_case(case, max_restart=0)
        U = torch.tensor(case.U, device="cuda")
        pn = ctx.select_degrees(U, var, nu_max, nu_min, p_min, p_max, eta_max_scope).cpu().numpy()
        ctx.close()
        hist.append(np.bincount(pn, minlength=p_max + 1)[1:].tolist())
        if np.array_equal(pn, p):
            break
        p = pn
    return p, hist


def adapt_step(case, ctx, U, nu_max=0.1, nu_min=0.001, p_min=1, p_max=5, var=1, reserve=None, eta_max_scope=1,
               fused=None):
    """One p-adaptation on the device: degrees from the indicator, criteria and
    face limiter (fr_select_degrees), a context for the new degree field (new
    degree buckets and face lists; ``reserve`` = the Context's max_restart /
    graphs, ``fused`` its launch mode), the state projected onto it
    (fr_project).  ``eta_max_scope``: the reading of the criteria's maximum
    indicator (1, the default: over the elements of the same degree; 0: over
    all elements, which on the isentropic vortex coarsens the vortex core to
    p <= 2 whatever p_max).
    Returns (new case description, new context, new state); when no degree
    changes these are the given case, context and state themselves."""
    import dataclasses

    from . import frx

    p_new = ctx.select_degrees(U, var, nu_max, nu_min, p_min, p_max, eta_max_scope).cpu().numpy()
    if np.array_equal(p_new.astype(np.int8), np.asarray(case.elem_p, np.int8)):
        return case, ctx, U
    new_case = dataclasses.replace(case, elem_p=p_new.astype(np.int8), U=None)
    new_ctx = frx.Context.from_case(new_case, fused=fused, **(reserve or {}))
    return new_case, new_ctx, ctx.project_to(U, new_ctx)
