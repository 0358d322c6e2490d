"""Time stepping through the library (paper_2606_11273_amd.dynamics.euler) against the oracle's.

tests/golden/dynamics_reference.npz holds 3 forward-Euler steps (dt = 0.05) of five unit disks
with seven close pairs (gaps 0.013 .. 0.103) under fixed N(0,1) forces and torques, by
oracle/dynamics.py at relative residual 1e-11 (written by
tests/golden/make_dynamics_reference.py, which calls only oracle/).  The library runs the same
steps in FP64 and mixed precision to 1e-10, each step from a new context (contacts, pair
precompute on the device) and the previous step's density as GMRES's initial guess.
Bars: the velocities of every step within max_i E^(i) <= 1e-5 (eq. rel_vel_err) and the
positions within 1e-6; the warm start needs fewer iterations than a cold start.
"""

import os

import numpy as np
import pytest

from oracle.system import rel_rigid_error
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

REF = os.path.join(os.path.dirname(__file__), "golden", "dynamics_reference.npz")


def test_euler_steps_match_oracle():
    from paper_2606_11273_amd import dynamics, native as nv
    ref = np.load(REF)
    dt, steps = float(ref["dt"]), int(ref["steps"])
    prm = nv.mfs_default_params()
    prm.delta_c = 0.2
    runs = {}
    for prec, warm in (("fp64", True), ("mixed", True), ("fp64", False)):
        r = dynamics.euler(ref["centers0"], 1.0, 36, 72, 0.7, ref["given"], dt, steps, precision=prec, tol=1e-10,
                           params=prm, warm_start=warm)
        runs[(prec, warm)] = r
        E = [rel_rigid_error(r["velocities"][s], ref["velocities"][s]).max() for s in range(steps)]
        dc = np.abs(r["centers"] - ref["centers"]).max()
        say(f"{prec} warm={warm}: iterations {r['iters']} (oracle {ref['iters'].tolist()}), pairs {r['n_pairs']}, "
            f"max E per step {np.array(E)}, max |c - c_ref| {dc:.1e}")
        assert max(E) <= 1e-5
        assert dc <= 1e-6
        assert np.abs(r["angles"] - ref["angles"]).max() <= 1e-6
    warm, cold = runs[("fp64", True)]["iters"], runs[("fp64", False)]["iters"]
    assert warm[0] == cold[0] and all(w < c for w, c in zip(warm[1:], cold[1:]))
