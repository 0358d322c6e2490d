"""Pins of the oracle's point sets (Sec. 3.3, Sec. 5, Sec. 6)."""

import json
import math
import os

import numpy as np

from oracle.geometry import (contacts, ellipse_points, fine_nodes, fine_sources, peanut_nodes, r_acc,
                             rigid_map, rigid_projector, ring_radius)
from oracle.params import MFSParams

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")


def test_default_parameters_are_the_papers():
    gold = json.load(open(GOLD))
    prm = MFSParams()
    for k in ("delta_c", "eps_ring", "n_fp", "n_ell", "m_p", "eps_trunc", "eps_trunc_fine", "gamma", "a_f",
              "mobius_r", "a_ell"):
        assert getattr(prm, k) == gold[k]["value"], k


def _invert(x, c):
    d = x - c
    return c + d / np.dot(d, d)


def test_r_acc_is_fixed_point_of_two_inversions():
    # Image accumulation point: successive reflections through the two unit
    # circles converge to c1 + R_acc e; it is a fixed point of the double inversion.
    for delta in (1e-4, 1e-3, 1e-2, 0.1, 0.5):
        c1 = np.array([0.0, 0.0])
        c2 = np.array([2.0 + delta, 0.0])
        p = c1 + np.array([r_acc(delta), 0.0])
        q = _invert(_invert(p, c2), c1)
        assert abs(q[0] - p[0]) < 1e-13 and abs(q[1]) < 1e-15
        # and it is the limit of iterating from the centre of disk 2
        z = c2.copy()
        for _ in range(20000):
            z = _invert(_invert(z, c1), c2)
        assert abs(_invert(z, c1)[0] - p[0]) < 1e-7


def test_ring_radius_rule():
    assert abs(ring_radius(150, 1e-12) - (1 - 12 * math.log(10) / 150)) < 1e-15


def test_ellipse_nodes_lie_on_ellipse_with_foci_0_and_a():
    prm = MFSParams()
    for delta in (1e-4, 1e-3, 1e-2, 0.03):
        z = ellipse_points(delta, prm)
        a = r_acc(delta)
        assert z.size > 0
        tip = a + prm.gamma * (1 - a)
        # sum of focal distances constant = major axis = tip - left end = 2 * (tip - a/2)
        major = 2 * (tip - a / 2)
        assert np.allclose(np.abs(z) + np.abs(z - a), major, rtol=0, atol=1e-13)
        assert np.all(np.abs(z) > ring_radius(prm.n_fp, prm.eps_ring))
        assert np.max(z.real) < tip + 1e-14 and np.max(np.abs(z)) < 1.0
    assert ellipse_points(0.1, prm).size == 0   # R_acc(0.1) < R_f: no enhancement


def test_fine_sources_and_nodes():
    prm = MFSParams()
    ci = np.array([1.0, -2.0])
    ang = 0.4
    ck = ci + 2.001 * np.array([math.cos(ang), math.sin(ang)])
    Yi, Yk = fine_sources(ci, ck, prm)
    n_enh = ellipse_points(0.001, prm).size
    assert Yi.shape[0] == Yk.shape[0] == prm.n_fp + n_enh
    # ellipse sources are mirror images through the midpoint
    assert np.allclose(Yi[prm.n_fp:] + Yk[prm.n_fp:], ci + ck, atol=1e-14)
    assert np.all(np.linalg.norm(Yi - ci, axis=1) < 1) and np.all(np.linalg.norm(Yk - ck, axis=1) < 1)
    Xi, Xk = fine_nodes(ci, ck, prm)
    assert Xi.shape == (180 + 400, 2) == Xk.shape
    assert np.allclose(np.linalg.norm(Xi - ci, axis=1), 1, atol=1e-14)
    # Moebius nodes are densest at the point facing the neighbour
    mob = Xi[180:]
    e = (ck - ci) / np.linalg.norm(ck - ci)
    cosang = (mob - ci) @ e
    near = np.sort(np.arccos(np.clip(cosang, -1, 1)))
    far = np.sort(np.arccos(np.clip(-(mob - ci) @ e, -1, 1)))
    assert near[1] - near[0] < 0.25 * (far[1] - far[0]) + 1e-12


def test_peanut_is_the_rolling_disk_clearance():
    # Every unit disk tangent to the pair (centre at distance 2 from one centre and
    # >= 2 from the other) touches the peanut: min distance centre-node = 1 within
    # the node spacing; no node lies inside either disk.
    for delta in (1e-3, 0.05, 0.2):
        ci = np.array([0.3, 0.1])
        ck = ci + (2 + delta) * np.array([math.cos(1.0), math.sin(1.0)])
        z = peanut_nodes(ci, ck, 400)
        d = 2 + delta
        psi = math.atan2(math.sqrt(4 - d * d / 4), d / 2)
        L = 6 * math.pi - 8 * psi
        steps = np.linalg.norm(np.diff(np.vstack([z, z[:1]]), axis=0), axis=1)
        assert np.all(steps <= L / 400 + 1e-12) and np.all(steps > 0.8 * L / 400)
        assert np.all(np.linalg.norm(z - ci, axis=1) > 1 - 1e-12)
        assert np.all(np.linalg.norm(z - ck, axis=1) > 1 - 1e-12)
        h = (L / 400) ** 2 / 2 + 1e-12
        for t in np.linspace(0, 2 * math.pi, 97):
            for c0, c1 in ((ci, ck), (ck, ci)):
                p = c0 + 2 * np.array([math.cos(t), math.sin(t)])
                if np.linalg.norm(p - c1) < 2 - 1e-12:
                    continue
                dmin = np.min(np.linalg.norm(z - p, axis=1))
                assert dmin > 1 - 1e-12 and dmin < 1 + 2 * h + (L / 400) ** 2


def test_rigid_projector_algebra():
    rng = np.random.default_rng(3)
    pts = rng.standard_normal((20, 2))
    K = rigid_map(pts, np.array([0.1, 0.2]))
    L = rigid_projector(K)
    assert np.allclose(L @ L, L, atol=1e-13) and np.allclose(L, L.T, atol=1e-14)
    assert np.allclose(K.T @ (np.eye(40) - L), 0, atol=1e-13)
    # K^T lambda: net force and torque of point forces lambda at pts about c
    lam = rng.standard_normal((20, 2))
    ft = K.T @ lam.reshape(-1)
    r = pts - np.array([0.1, 0.2])
    assert np.allclose(ft[:2], lam.sum(0)) and abs(ft[2] - np.sum(r[:, 0] * lam[:, 1] - r[:, 1] * lam[:, 0])) < 1e-13


def test_contacts_brute_force():
    rng = np.random.default_rng(4)
    c = rng.uniform(0, 20, (300, 2))
    a = np.ones(300)
    pr = contacts(c, a, 0.2)
    ref = [(i, k) for i in range(300) for k in range(i + 1, 300) if np.linalg.norm(c[i] - c[k]) <= 2.2]
    assert [tuple(p) for p in pr] == ref
