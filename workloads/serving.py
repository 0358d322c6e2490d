"""Seeded request streams for the serving workload: independent mobility solves.

Request k of a stream with seed s: P ~ U{P_lo..P_hi}, area fraction ~ U[0.4, 0.65],
min gap = 10^U[-4, -2], a perturbed triangular lattice relaxed to that gap (the
generator of the P = 1000 and P = 10^4 workloads), N_c = 36 sources on radius 0.7,
M_c = 72 nodes, forces and torques ~ N(0,1) with zero net force.  Arrivals are a
Poisson process: exponential gaps of mean 1/rate.  Geometry and random draws only.
"""

from __future__ import annotations

import numpy as np

from .packings import lattice_packing
from .rhs import mobility_rhs

SERVING_SEED_BASE = 260611273 + 4000
_RHO_SERVING = 0.9


def serving_request(k, seed=SERVING_SEED_BASE, P_lo=50, P_hi=3000):
    """Request k of the stream: dict(centers, radii, n_src, n_col, r_src, given, P, phi, g_min, seed)."""
    rng = np.random.default_rng([seed, k])
    P = int(rng.integers(P_lo, P_hi + 1))
    phi = float(rng.uniform(0.4, 0.65))
    g_min = float(10.0 ** rng.uniform(-4.0, -2.0))
    s = int(rng.integers(0, 2**31 - 1))
    c, a, _ = lattice_packing(s, P, phi, g_min, _RHO_SERVING)
    return dict(centers=np.ascontiguousarray(c, dtype=np.float64), radii=np.ascontiguousarray(a, dtype=np.float64),
                n_src=np.full(P, 36, dtype=np.int32), n_col=np.full(P, 72, dtype=np.int32),
                r_src=np.full(P, 0.7), given=mobility_rhs(s, P), P=P, phi=phi, g_min=g_min, seed=s)


def poisson_arrivals(n, rate, seed=SERVING_SEED_BASE):
    """Arrival times (seconds from 0) of n requests at mean rate `rate` per second."""
    rng = np.random.default_rng([seed, 10**6])
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
