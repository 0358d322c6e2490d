"""Time stepping of rigid disks under given forces and torques (oracle).

Test infrastructure: a plain FP64 reference for the library's time-stepping driver; only
tests, the smoke check and the benchmark's CPU baseline use it.

The method's application is the motion of dense suspensions (Sec. 1), advanced in time by
one mobility solve per step; the paper fixes no integrator.  This oracle takes forward
Euler: at step s the mobility problem (Alg. 2 with the mobility projections of Sec. 4.4)
is solved for the configuration c_s under the forces and torques g_s, giving [v; omega],
and then c_{s+1} = c_s + dt v, theta_{s+1} = theta_s + dt omega.  The disks' coarse and
fine discretisations do not turn with them (a disk is a circle), so theta only records
the rotation.
"""

from __future__ import annotations

import numpy as np

from .params import MFSParams
from .system import System, solve


def euler(centers, radii, n_src, n_col, r_src, given, dt, steps, tol, prm=MFSParams(), maxit=500):
    """Forward Euler over `steps` steps.  given: (P, 3) forces and torques, or a function
    (step, centers) -> (P, 3).  Returns dict of centers (steps + 1, P, 2), angles
    (steps + 1, P), velocities (steps, P, 3) and GMRES iterations per step."""
    c = np.array(centers, dtype=np.float64).reshape(-1, 2)
    P = c.shape[0]
    th = np.zeros(P)
    cs, ths, vs, its = [c.copy()], [th.copy()], [], []
    for s in range(steps):
        g = np.asarray(given(s, c) if callable(given) else given, dtype=np.float64).reshape(P, 3)
        S = System(c, radii, n_src, n_col, r_src, "mobility", prm)
        out, _, info = solve(S, g, tol, maxit)
        c = c + dt * out[:, :2]
        th = th + dt * out[:, 2]
        cs.append(c.copy())
        ths.append(th.copy())
        vs.append(out.copy())
        its.append(int(info["iters"]))
    return dict(centers=np.stack(cs), angles=np.stack(ths), velocities=np.stack(vs), iters=its)
