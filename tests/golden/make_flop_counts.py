"""Writes flop_counts.json: the floating-point operations of the method per
degree of freedom, counted operation by operation on the oracle's own
residual (oracle.Oracle.count_flops: counted reals for the residual, counted
forward-mode dual numbers for the residual with its tangent).  These counts are
the work model of the measured kernels' rooflines.

Counted on
  * uniform-degree periodic Navier-Stokes boxes (4x4x4 elements, p = 1..5),
    where every face is conforming;
  * a 4x128x8 slab (every 32nd x column, closed periodically in x) of the
    128x128x8 Re 60000 workload with its i.i.d. degrees p in {1,2,3,4}
    (weights .3/.3/.25/.15), mortar faces included; the per-DOF counts apply
    to the whole workload, whose degree field has the same distribution.

Calls only oracle/ and the seeded input generators.  Run from the repository
root: python tests/golden/make_flop_counts.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1910_03693_amd import inputs as I  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "flop_counts.json")


def uniform_box(p):
    return I.case_ns_mixed(4, 4, 4, k=90, lengths=(1.0, 1.0, 1.0), pvals=(p,), pw=(1,), re=3900.0, ma=0.2)


def slab(case, nx_slab):
    """The first nx_slab x columns of a structured box case, closed
    periodically in x (elements, degrees and state kept)."""
    nx, ny, nz = case.mesh["shape"]
    sel = np.nonzero(np.arange(case.mesh["n_elem"]) % nx < nx_slab)[0]
    L = case.mesh["lengths"]
    m = I.box_mesh(nx_slab, ny, nz, (L[0] * nx_slab / nx, L[1], L[2]))
    m["elem_xyz"] = case.mesh["elem_xyz"][sel]
    off = I.sp_offsets(case.elem_p)
    cols = np.concatenate([np.arange(off[e], off[e + 1]) for e in sel])
    return I.Case("slab", m, case.elem_p[sel].copy(), np.ascontiguousarray(case.U[:, cols]), case.physics,
                  case.flux, case.gamma, case.mu, case.prandtl, case.farfield, {})


def counts(case, seed):
    orc = oracle.Oracle.from_case(case)
    v = I.random_direction(case.U.size, seed).reshape(case.U.shape)
    fr, _ = orc.count_flops(case.U)
    fd, _ = orc.count_flops(case.U, v)
    n = case.U.size
    return {"dof": int(n), "residual_flops": fr, "dual_flops": fd,
            "residual_per_dof": round(fr / n, 3), "dual_per_dof": round(fd / n, 3)}


def main():
    out = {"source": "operation counts of the oracle's residual on counted scalars: one per +, -, *, / and "
                     "square root; forward-mode dual arithmetic at its own cost (oracle.Oracle.count_flops)",
           "uniform_4x4x4_navier_stokes": {}}
    for p in range(1, 6):
        out["uniform_4x4x4_navier_stokes"][str(p)] = counts(uniform_box(p), 4100 + p)
        print("p", p, out["uniform_4x4x4_navier_stokes"][str(p)], flush=True)
    sub = slab(I.config(5), 4)
    out["navier_stokes_128x128x8_slab_4x128x8"] = counts(sub, 4005)
    out["navier_stokes_128x128x8_slab_4x128x8"]["degree_histogram_p1_to_p4"] = \
        np.bincount(sub.elem_p, minlength=5)[1:].tolist()
    print("slab", out["navier_stokes_128x128x8_slab_4x128x8"], flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
