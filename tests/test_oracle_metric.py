"""Pins of the error metric of eq. rel_vel_err (Sec. 6.2), which every parity assertion uses.

E^(i) = (|v_i - v_ref,i|_2 + |omega_i - omega_ref,i|) / max_j (|v_ref,j|_2 + |omega_ref,j|): the
error of body i against the largest rigid-body speed of the reference.  Hand-computed values
on a two-body case fix the 2-norm of the translational part, the absolute rotational part,
the normalisation by the reference (not the tested solution) and by its largest body (not
the body itself).  The benchmark's copy (bench.rel_rigid_error, the maximum over bodies) is
pinned to the same values.
"""

import math

import numpy as np

import bench
from oracle.system import rel_rigid_error

REF = np.array([[1.0, 0.0, 0.5], [3.0, 4.0, 0.0]])     # speeds s = 1 + 0.5 = 1.5 and 5 + 0 = 5
OUT = np.array([[1.0, 0.0, 0.0], [0.0, 2.0, 1.0]])


def test_hand_computed_values():
    e = rel_rigid_error(OUT, REF)
    # body 0: (|(0, 0)| + |0 - 0.5|) / 5; body 1: (|(-3, -2)| + |1 - 0|) / 5
    assert np.allclose(e, [0.5 / 5, (math.sqrt(13.0) + 1.0) / 5], rtol=0, atol=1e-15)
    assert bench.rel_rigid_error(OUT, REF) == e.max()


def test_reference_side_and_invariances():
    # normalised by the reference's speeds: swapping the arguments changes the value
    assert not np.allclose(rel_rigid_error(REF, OUT), rel_rigid_error(OUT, REF))
    # OUT as the reference: speeds 1 and |(0, 2)| + 1 = 3
    assert np.allclose(rel_rigid_error(REF, OUT), [0.5 / 3, (math.sqrt(13.0) + 1.0) / 3], rtol=0, atol=1e-15)
    # a common scale of both solutions leaves it unchanged; an exact solution gives zero
    assert np.allclose(rel_rigid_error(7.0 * OUT, 7.0 * REF), rel_rigid_error(OUT, REF), rtol=1e-15, atol=0)
    assert np.all(rel_rigid_error(REF, REF) == 0.0)
    # the sign of the rotation counts, not only its size
    flip = REF.copy()
    flip[0, 2] = -0.5
    assert math.isclose(rel_rigid_error(flip, REF)[0], 1.0 / 5.0, rel_tol=1e-15)
