"""The work model of the rooflines: floating-point operation counts of the
oracle's residual on counted scalars (tests/golden/flop_counts.json, written by
tests/golden/make_flop_counts.py).  Pins: the counted evaluations return the
oracle's own residual bit for bit and a tangent equal to the complex-step one;
the counts are exactly proportional to the number of elements of a uniform
periodic mesh; a dual operation costs between two and four real ones; and the
stored table is what the oracle counts now."""
import json
import os

import numpy as np
import pytest

from paper_1910_03693_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "flop_counts.json")


def _box(nx, p):
    return I.case_ns_mixed(nx, 4, 4, k=90, lengths=(nx / 4.0, 1.0, 1.0), pvals=(p,), pw=(1,), re=3900.0, ma=0.2)


@pytest.mark.parametrize("p", [1, 3])
def test_counted_evaluations_are_the_oracle(oracle_mod, p):
    case = _box(4, p)
    orc = oracle_mod.Oracle.from_case(case)
    v = I.random_direction(case.U.size, 4100 + p).reshape(case.U.shape)
    f0, R = orc.count_flops(case.U)
    f1, J = orc.count_flops(case.U, v)
    assert np.array_equal(R.ravel(), orc.residual(case.U).ravel())
    Jc = orc.jvp(case.U, v).ravel()
    assert np.abs(J.ravel() - Jc).max() <= 1e-13 * np.abs(Jc).max()
    assert 2.0 * f0 <= f1 <= 4.0 * f0


def test_counts_scale_with_the_mesh(oracle_mod):
    f = []
    for nx in (4, 8):
        case = _box(nx, 2)
        f.append(oracle_mod.Oracle.from_case(case).count_flops(case.U)[0])
    assert f[1] == 2 * f[0]


def test_stored_table_is_the_oracle_count(oracle_mod):
    with open(GOLDEN) as fh:
        table = json.load(fh)
    for p in range(1, 6):
        case = _box(4, p)
        orc = oracle_mod.Oracle.from_case(case)
        v = I.random_direction(case.U.size, 4100 + p).reshape(case.U.shape)
        row = table["uniform_4x4x4_navier_stokes"][str(p)]
        assert orc.count_flops(case.U)[0] == row["residual_flops"]
        assert orc.count_flops(case.U, v)[0] == row["dual_flops"]
    slab = table["navier_stokes_128x128x8_slab_4x128x8"]
    assert slab["residual_per_dof"] > table["uniform_4x4x4_navier_stokes"]["1"]["residual_per_dof"]
