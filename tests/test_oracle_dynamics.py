"""Pins of the time-stepping oracle (oracle/dynamics.py, forward Euler on mobility solves).

* a single disk under a force and a torque moves with the closed-form velocity
  v = F (1/2 - ln a) / (4 pi mu), omega = t / (4 pi mu a^2) at every step, so after s steps
  c_s = c_0 + s dt v and theta_s = s dt omega;
* translating the initial configuration translates every later one (the method has no
  preferred origin), on three disks with one close pair, over two steps;
* halving dt halves the difference from a finer solution at the same time (first order).
"""

import math

import numpy as np

from oracle.dynamics import euler
from oracle.params import MFSParams

SMALL = MFSParams(n_fp=60, n_ell=30, m_p=100)   # cheap fine grids


def test_single_disk_moves_with_the_closed_form_velocity():
    a, mu = 1.2, 1.7
    ft = np.array([[0.4, -1.1, 0.7]])
    r = euler(np.array([[0.3, -0.2]]), a, 36, 72, 0.7, ft, 0.25, 3, 1e-13, MFSParams(mu=mu))
    v = ft[0, :2] * (0.5 - math.log(a)) / (4 * math.pi * mu)
    w = ft[0, 2] / (4 * math.pi * mu * a * a)
    for s in range(4):
        assert np.allclose(r["centers"][s, 0], [0.3, -0.2] + s * 0.25 * v, rtol=0, atol=1e-12)
        assert abs(r["angles"][s, 0] - s * 0.25 * w) < 1e-12


def _three():
    c = np.array([[0.0, 0.0], [2.05, 0.1], [0.4, 2.6]])
    g = np.array([[0.5, 0.2, 0.3], [-0.5, 0.1, -0.2], [0.0, -0.3, 0.4]])
    return c, g


def test_translation_covariance():
    c, g = _three()
    r1 = euler(c, 1.0, 36, 72, 0.7, g, 0.2, 2, 1e-12, SMALL)
    shift = np.array([11.5, -4.25])
    r2 = euler(c + shift, 1.0, 36, 72, 0.7, g, 0.2, 2, 1e-12, SMALL)
    assert np.abs(r2["centers"] - shift - r1["centers"]).max() < 1e-9
    assert np.abs(r2["angles"] - r1["angles"]).max() < 1e-9
    assert np.abs(r1["centers"][-1] - c).max() > 1e-3          # the disks did move


def test_first_order_in_dt():
    c, g = _three()
    T = 0.4
    end = {n: euler(c, 1.0, 36, 72, 0.7, g, T / n, n, 1e-12, SMALL)["centers"][-1] for n in (1, 2, 4)}
    e1 = np.abs(end[1] - end[4]).max()
    e2 = np.abs(end[2] - end[4]).max()
    # Euler's error is c1 dt + O(dt^2): e(dt) - e(dt/4) over e(dt/2) - e(dt/4) tends to 3
    assert 2.0 < e1 / e2 < 4.0, (e1, e2)
