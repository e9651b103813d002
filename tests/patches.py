"""Element patches for sampled parity checks at full size.

The residual (and its tangent) at the solution points of an element depends
only on the state of that element and of its face neighbours: the common
solution, BR2 gradients and common fluxes of a face use the two sides' traces
of q and of the uncorrected gradient, and each side's traces come from its own
state alone.  A patch made of the element and its face neighbours, with every
other face of the neighbours closed by a wall, therefore reproduces the
element's residual block of the full mesh.  Here a patch is built by pure
gathering (no arithmetic of the method); tests pin the construction against
the oracle's full-mesh residual on the CPU.
"""
from __future__ import annotations

import numpy as np

from paper_1910_03693_amd import inputs as I


def patch_ids(elem_nbr, e):
    ids = [int(e)]
    for f in range(6):
        nb = int(elem_nbr[e, f])
        if nb >= 0 and nb not in ids:
            ids.append(nb)
    return ids


def patch_case(case, e, offsets=None):
    """Case made of element e (patch element 0) and its face neighbours."""
    nbr = case.mesh["elem_nbr"]
    ids = patch_ids(nbr, e)
    loc = {g: i for i, g in enumerate(ids)}
    pn = np.full((len(ids), 6), I.BC_WALL, np.int32)
    for i, g in enumerate(ids):
        for f in range(6):
            nb = int(nbr[g, f])
            if nb < 0:
                pn[i, f] = nb
            elif i == 0:
                pn[i, f] = loc[nb]
            elif nb == e:
                pn[i, f] = 0
    off = I.sp_offsets(case.elem_p) if offsets is None else offsets
    cols = np.concatenate([np.arange(off[g], off[g + 1]) for g in ids])
    mesh = {"elem_xyz": case.mesh["elem_xyz"][ids], "elem_nbr": pn, "n_elem": len(ids)}
    sub = I.Case(case.name + f"_patch{e}", mesh, case.elem_p[ids].copy(), case.U[:, cols].copy(), case.physics,
                 case.flux, case.gamma, case.mu, case.prandtl, case.farfield, dict(case.extra))
    return sub, cols


def element_block(case, e, offsets=None):
    off = I.sp_offsets(case.elem_p) if offsets is None else offsets
    return np.arange(off[e], off[e + 1])


def sample_elements(elem_p, per_degree, seed):
    rng = np.random.default_rng(seed)
    out = []
    for p in np.unique(elem_p):
        idx = np.nonzero(elem_p == p)[0]
        out.extend(rng.choice(idx, size=min(per_degree, idx.size), replace=False).tolist())
    return sorted(out)
