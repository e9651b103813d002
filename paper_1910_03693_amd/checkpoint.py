"""Checkpoint and resume of a solution: the degree field and the state, with
the mesh description, in a NumPy archive (no pickled objects)."""
from __future__ import annotations

import numpy as np


def save(path, case, U, t=0.0, step=0):
    """U: the state as a host array or a device tensor, in the layout of
    case.elem_p."""
    if hasattr(U, "detach"):
        U = U.detach().cpu().numpy()
    np.savez(path, elem_xyz=case.mesh["elem_xyz"], elem_nbr=case.mesh["elem_nbr"], elem_p=case.elem_p,
             U=np.asarray(U, dtype=np.float64), t=np.float64(t), step=np.int64(step),
             gas=np.array([case.physics, case.flux, case.gamma, case.mu, case.prandtl], dtype=np.float64),
             farfield=case.farfield)


def load(path, name="restart"):
    """Returns (case, t, step); case.U holds the saved state."""
    from .inputs import Case

    with np.load(path, allow_pickle=False) as z:
        g = z["gas"]
        mesh = {"elem_xyz": z["elem_xyz"], "elem_nbr": z["elem_nbr"], "n_elem": int(z["elem_p"].size)}
        case = Case(name, mesh, z["elem_p"].astype(np.int8), z["U"].copy(), int(g[0]), int(g[1]), float(g[2]),
                    float(g[3]), float(g[4]), z["farfield"].copy(), {})
        return case, float(z["t"]), int(z["step"])
