"""Write tests/golden/dynamics_reference.npz: forward-Euler motion of five disks by the oracle.

Five unit disks (N_c = 36 on radius 0.7, M_c = 72, the paper's fine discretisation, contact
threshold 0.2) with seven close pairs at gaps 0.013 .. 0.103, under fixed forces and torques
drawn from N(0,1) (net force removed), are moved for 3 steps of dt = 0.05 by
oracle/dynamics.py: one mobility solve (Alg. 2, Sec. 4.4) to relative residual 1e-11 per
step, then c += dt v, theta += dt omega.  Only oracle/ is used.

Run from the repository root:  python tests/golden/make_dynamics_reference.py
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.dynamics import euler  # noqa: E402
from oracle.params import MFSParams  # noqa: E402

CENTERS = np.array([[0.0, 0.0], [2.03, 0.05], [1.0, 1.78], [-1.05, 1.8], [3.1, 1.86]])
DT, STEPS, TOL = 0.05, 3, 1e-11


def given():
    g = np.random.default_rng(2606).standard_normal((5, 3))
    g[:, :2] -= g[:, :2].mean(0)
    return g


def main():
    t0 = time.time()
    g = given()
    r = euler(CENTERS, 1.0, 36, 72, 0.7, g, DT, STEPS, TOL, MFSParams())
    print(f"{STEPS} steps in {time.time() - t0:.1f} s, iterations {r['iters']}")
    np.savez(os.path.join(ROOT, "tests", "golden", "dynamics_reference.npz"), centers0=CENTERS, given=g, dt=DT,
             steps=STEPS, tol=TOL, centers=r["centers"], angles=r["angles"], velocities=r["velocities"],
             iters=np.array(r["iters"]))


if __name__ == "__main__":
    main()
