"""Time stepping of rigid disks under given forces and torques, one mobility solve per step.

The method's application is the motion of dense suspensions (Sec. 1); the paper fixes no
integrator, so this driver takes forward Euler: at step s the library solves the mobility
problem (Alg. 2, Sec. 4.4) for the configuration c_s under the forces and torques g_s and
moves every disk by dt [v; omega].  Each step builds a context for the new positions (contact
list, clusters and the pair precompute of the new close pairs on the device) and starts GMRES
from the previous step's density (the unknown lives on nodes that move with their disks, so
the last solution is a close initial guess).  The disks' discretisations do not turn with
them (a disk is a circle); theta only records the rotation.

Every computation runs in the library; this module sequences its calls.
"""

from __future__ import annotations

import time

import numpy as np
import torch

from . import native as nv


def euler(centers, radii, n_src, n_col, r_src, given, dt, steps, precision="mixed", tol=1e-9, max_iter=500,
          params=None, warm_start=True, callback=None):
    """Forward Euler over `steps` steps.

    given: (P, 3) forces and torques, or a function (step, centers) -> (P, 3).
    Returns a dict of centers (steps + 1, P, 2), angles (steps + 1, P), velocities
    (steps, P, 3), and per step the GMRES iterations, refinement steps, close pairs and
    seconds.  A step whose disks overlap raises the library's MFSError (MFS_ERR_GEOMETRY):
    choose dt so that the gaps stay open."""
    c = np.array(centers, dtype=np.float64).reshape(-1, 2)
    P = c.shape[0]
    radii = np.broadcast_to(np.asarray(radii, dtype=np.float64), (P,)).copy()
    n_src = np.broadcast_to(np.asarray(n_src, dtype=np.int32), (P,)).copy()
    n_col = np.broadcast_to(np.asarray(n_col, dtype=np.int32), (P,)).copy()
    r_src = np.broadcast_to(np.asarray(r_src, dtype=np.float64), (P,)).copy()
    th = np.zeros(P)
    out = dict(centers=[c.copy()], angles=[th.copy()], velocities=[], iters=[], outer=[], n_pairs=[], seconds=[])
    mu = None
    for s in range(steps):
        t0 = time.perf_counter()
        g = np.asarray(given(s, c) if callable(given) else given, dtype=np.float64).reshape(P, 3)
        ctx = nv.mfs_setup(c, radii, n_src, n_col, r_src, params)
        try:
            n_pairs = nv.mfs_precompute_pairs(ctx, "mobility")
            x0 = mu if (warm_start and mu is not None) else None
            vel, info = nv.mfs_gmres_solve(ctx, "mobility", precision, g, tol, max_iter, x0=x0)
            if mu is None:
                _, _, Nt, _ = nv.mfs_get_sizes(ctx)
                mu = torch.zeros(2 * Nt, dtype=torch.float64, device="cuda")
            nv.mfs_get_density(ctx, 0, mu)
            torch.cuda.synchronize()
        finally:
            nv.mfs_destroy(ctx)
        c = c + dt * vel[:, :2]
        th = th + dt * vel[:, 2]
        out["centers"].append(c.copy())
        out["angles"].append(th.copy())
        out["velocities"].append(vel.copy())
        out["iters"].append(info["iters"])
        out["outer"].append(info["outer"])
        out["n_pairs"].append(int(n_pairs))
        out["seconds"].append(time.perf_counter() - t0)
        if callback is not None:
            callback(s, c, vel, info)
    for key in ("centers", "angles", "velocities"):
        out[key] = np.stack(out[key])
    return out
