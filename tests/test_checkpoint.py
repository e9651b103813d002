"""Checkpoint round trip (CPU): degree field, state and mesh come back
unchanged, through an archive that needs no pickling."""
import numpy as np

from paper_1910_03693_amd import checkpoint
from paper_1910_03693_amd import inputs as I


def test_round_trip(tmp_path):
    case = I.case_ns_mixed(3, 3, 2, k=81, lengths=(1.0, 1.0, 0.6), wall=True, pvals=(1, 2, 3), pw=(1, 1, 1))
    p = tmp_path / "state.npz"
    checkpoint.save(p, case, case.U, t=0.25, step=5)
    back, t, step = checkpoint.load(p)
    assert t == 0.25 and step == 5
    assert np.array_equal(back.elem_p, case.elem_p)
    assert np.array_equal(back.U, case.U)
    assert np.array_equal(back.mesh["elem_nbr"], case.mesh["elem_nbr"])
    assert np.array_equal(back.mesh["elem_xyz"], case.mesh["elem_xyz"])
    assert (back.physics, back.flux, back.gamma, back.mu, back.prandtl) == (case.physics, case.flux, case.gamma,
                                                                            case.mu, case.prandtl)
    assert np.array_equal(back.farfield, case.farfield)
    with np.load(p, allow_pickle=False) as z:
        assert all(z[k].dtype != object for k in z.files)
