"""Pins of the oracle's one-body solves, RHS and post-processing (Sec. 3.1, Sec. 4.1).

Single disk of radius a in a fluid of viscosity mu (w = 0 frame of Remark 1):
* torque t: rotation omega = t / (4 pi mu a^2) and the rotlet exterior field
  t/(4 pi mu) (x - c)^perp / |x - c|^2;
* force F: translation v = F (1/2 - ln a) / (4 pi mu) (Stokeslet plus potential
  dipole; it degenerates at a = sqrt(e), the case named in Remark 1).
Resistance inverts these maps.
"""

import math

import numpy as np

from oracle.kernel import direct_sum
from oracle.onebody import one_body
from oracle.params import MFSParams
from oracle.system import System, solve


def _closed(a, mu, ft):
    v = ft[:2] * (0.5 - math.log(a)) / (4 * math.pi * mu)
    return np.array([v[0], v[1], ft[2] / (4 * math.pi * mu * a * a)])


def test_single_disk_mobility_closed_forms():
    for a, mu in ((1.0, 1.0), (1.4, 1.0), (1.0, 2.5)):
        prm = MFSParams(mu=mu)
        S = System(np.array([[0.3, -0.7]]), a, 36, 72, 0.7, "mobility", prm)
        for ft in (np.array([0.0, 0.0, 1.0]), np.array([1.0, -0.4, 0.0]), np.array([0.3, 0.9, -2.0])):
            out, _, _ = solve(S, ft[None], 1e-13)
            assert np.max(np.abs(out[0] - _closed(a, mu, ft))) < 1e-10 * np.max(np.abs(_closed(a, mu, ft)))


def test_single_disk_resistance_closed_forms():
    for a, mu in ((1.0, 1.0), (1.4, 2.0)):
        prm = MFSParams(mu=mu)
        S = System(np.array([[-1.0, 2.0]]), a, 36, 72, 0.7, "resistance", prm)
        vw = np.array([0.2, -0.5, 0.8])
        out, _, _ = solve(S, vw[None], 1e-13)
        f = vw[:2] * 4 * math.pi * mu / (0.5 - math.log(a))
        t = vw[2] * 4 * math.pi * mu * a * a
        ref = np.array([f[0], f[1], t])
        assert np.max(np.abs(out[0] - ref)) < 1e-9 * np.max(np.abs(ref))


def test_torqued_disk_exterior_field_is_rotlet():
    prm = MFSParams()
    c = np.array([0.5, 0.25])
    S = System(c[None], 1.0, 36, 72, 0.7, "mobility", prm)
    t = 1.3
    out, mu, _ = solve(S, np.array([[0.0, 0.0, t]]), 1e-13)
    ob = S.cls[0]
    lam_bar = ob.pinv(mu)
    lam0 = ob.K @ np.linalg.solve(ob.K.T @ ob.K, np.array([0.0, 0.0, t]))
    sig = ob.project(lam_bar) + lam0
    x = c + np.array([[1.5, 0.0], [0.0, -2.0], [3.0, 3.0], [1.02, 0.1]])
    u = direct_sum(x, S.Y, sig.reshape(-1, 2))
    d = x - c
    ref = t / (4 * math.pi) * np.stack([-d[:, 1], d[:, 0]], axis=1) / np.sum(d * d, axis=1)[:, None]
    err = np.max(np.abs(u - ref), axis=1)
    assert np.all(err[:3] < 1e-12)          # well outside the disk: exact to rounding
    assert err[3] < 1e-6                    # 0.02 outside the boundary: MFS accuracy


def test_one_body_algebra():
    ob = one_body(1.0, 36, 72, 0.7, 1.0, "mobility", 1e-14)
    assert ob.s.size == 72                                  # S_L has full column rank
    assert np.allclose(ob.K.T @ ob.IL, 0, atol=1e-13)       # K^T (I - L) = 0
    IL2 = ob.IL @ ob.IL
    assert np.allclose(IL2, ob.IL, atol=1e-13)
    # S_L^+ of rigid data B w is K (K^T K)^{-1} w exactly (S_L K = B K^T K)
    w = np.array([0.3, -1.2, 0.7])
    lam = ob.pinv(ob.B @ w)
    assert np.allclose(lam, ob.K @ np.linalg.solve(ob.K.T @ ob.K, w), atol=1e-10)
    assert np.allclose(-ob.K.T @ lam, -w, atol=1e-10)
    rb = one_body(1.0, 36, 72, 0.7, 1.0, "resistance", 1e-14)
    # resistance pseudoinverse reproduces data in the range of P
    lam = np.random.default_rng(0).standard_normal(72)
    assert np.allclose(rb.pinv(rb.P @ lam), lam, atol=1e-7 * np.linalg.norm(lam))
