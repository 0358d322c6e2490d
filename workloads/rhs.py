"""Seeded right-hand-side draws (forces/torques or rigid velocities per body).

Sec. 6.1 samples the prescribed quantities from a standard normal distribution
and shifts the forces so that they sum to zero; Fig. 1 drives every disk by a
unit torque.  Arrays are (P, 3) with columns (x, y, rotational).
"""

from __future__ import annotations

import numpy as np


def mobility_rhs(seed, P, zero_net_force=True):
    """Forces and torques ~ N(0,1); forces shifted so that sum f = 0."""
    rng = np.random.default_rng(seed + 7)
    ft = rng.standard_normal((P, 3))
    if zero_net_force:
        ft[:, :2] -= ft[:, :2].mean(axis=0, keepdims=True)
    return ft


def resistance_rhs(seed, P):
    """Translational and angular velocities ~ N(0,1)."""
    rng = np.random.default_rng(seed + 11)
    return rng.standard_normal((P, 3))


def unit_torques(P):
    """Zero force and unit torque on every body."""
    ft = np.zeros((P, 3))
    ft[:, 2] = 1.0
    return ft
