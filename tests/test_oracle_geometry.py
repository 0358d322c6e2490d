"""Pins of the oracle's point sets (Sec. 3.3, Sec. 5, Sec. 6)."""

import json
import math
import os

import numpy as np

from oracle.geometry import (contacts, ellipse_points, fine_count, fine_nodes, fine_sources, limit_point,
                             peanut_nodes, r_acc, rigid_map, rigid_projector, ring_radius)
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


# -- unequal radii (the bidisperse workload; a reading of the paper) ---------------------------------------

def _invert_r(p, c, r):
    v = p - c
    return c + r * r * v / (v @ v)


def test_limit_point_is_fixed_by_both_inversions():
    # x1 inside disk 1 (radius a1 at the origin) is the common fixed point of the inversions
    # in both circles: inverting in circle 1 and then in circle 2 returns it.
    for a1, a2 in ((1.0, 1.4), (1.4, 1.0), (1.0, 1.0), (1.4, 1.4)):
        for delta in (1e-4, 1e-2, 0.15):
            d = a1 + a2 + delta
            p = np.array([limit_point(a1, a2, d), 0.0])
            q = _invert_r(_invert_r(p, np.zeros(2), a1), np.array([d, 0.0]), a2)
            assert abs(q[0] - p[0]) < 1e-12 * max(1.0, d) and 0 < p[0] < a1
            if a1 == a2 == 1.0:
                assert abs(p[0] - r_acc(delta)) < 1e-14


def test_unequal_ellipse_and_fine_sets():
    prm = MFSParams()
    assert fine_count(1.0, prm) == 150 and fine_count(1.4, prm) == 210
    ci = np.array([0.2, -1.0])
    ang = -0.7
    e = np.array([math.cos(ang), math.sin(ang)])
    for ai, ak in ((1.0, 1.4), (1.4, 1.0)):
        delta = 2e-3
        ck = ci + (ai + ak + delta) * e
        for a1, a2, c0, sgn in ((ai, ak, ci, 1), (ak, ai, ck, -1)):
            z = ellipse_points(delta, prm, a1, a2)
            x1 = limit_point(a1, a2, ai + ak + delta)
            major = x1 + 2 * prm.gamma * (a1 - x1)
            assert z.size > 0
            assert np.allclose(np.abs(z) + np.abs(z - x1), major, rtol=0, atol=1e-13)
            assert np.all(np.abs(z) > a1 * ring_radius(fine_count(a1, prm), prm.eps_ring))
        Yi, Yk = fine_sources(ci, ck, prm, ai, ak)
        ni, nk = fine_count(ai, prm), fine_count(ak, prm)
        assert Yi.shape[0] == ni + ellipse_points(delta, prm, ai, ak).size
        assert Yk.shape[0] == nk + ellipse_points(delta, prm, ak, ai).size
        assert np.all(np.linalg.norm(Yi - ci, axis=1) < ai) and np.all(np.linalg.norm(Yk - ck, axis=1) < ak)
        # ellipse sources lie on the centre line, toward the neighbour
        assert np.all((Yi[ni:] - ci) @ e > 0) and np.all((Yk[nk:] - ck) @ e < 0)
        Xi, Xk = fine_nodes(ci, ck, prm, ai, ak)
        assert Xi.shape[0] == math.ceil(1.2 * ni) + 400 and Xk.shape[0] == math.ceil(1.2 * nk) + 400
        assert np.allclose(np.linalg.norm(Xi - ci, axis=1), ai, atol=1e-13)
        assert np.allclose(np.linalg.norm(Xk - ck, axis=1), ak, atol=1e-13)


def test_unequal_peanut_is_the_rolling_disk_clearance():
    # The rolling unit circle touching both disks touches the peanut from outside: every
    # unit disk tangent to one body and not overlapping the other keeps distance >= 1 from
    # the peanut nodes; no node is inside a body; nodes are uniform in arc length.
    for ai, ak in ((1.0, 1.4), (1.4, 1.0), (1.4, 1.4)):
        for delta in (1e-3, 0.05):
            ci = np.array([0.3, 0.1])
            ck = ci + (ai + ak + delta) * np.array([math.cos(1.0), math.sin(1.0)])
            z = peanut_nodes(ci, ck, 400, ai, ak)
            # perimeter: two disk arcs and two arcs of the rolling unit circle, whose centre
            # is at distances ai + 1 and ak + 1 from the centres (law of cosines for the angles)
            d = ai + ak + delta
            psi_i = math.acos(((ai + 1) ** 2 + d * d - (ak + 1) ** 2) / (2 * (ai + 1) * d))
            psi_k = math.acos(((ak + 1) ** 2 + d * d - (ai + 1) ** 2) / (2 * (ak + 1) * d))
            L = 2 * ai * (math.pi - psi_i) + 2 * ak * (math.pi - psi_k) + 2 * (math.pi - psi_i - psi_k)
            steps = np.linalg.norm(np.diff(np.vstack([z, z[:1]]), axis=0), axis=1)
            assert np.all(steps <= L / 400 + 1e-12) and np.all(steps > 0.8 * L / 400)
            assert abs(steps.sum() - L) < 1e-3 * L
            assert np.all(np.linalg.norm(z - ci, axis=1) > ai - 1e-12)
            assert np.all(np.linalg.norm(z - ck, axis=1) > ak - 1e-12)
            for t in np.linspace(0, 2 * math.pi, 97):
                for c0, r0, c1, r1 in ((ci, ai, ck, ak), (ck, ak, ci, ai)):
                    p = c0 + (r0 + 1) * np.array([math.cos(t), math.sin(t)])
                    if np.linalg.norm(p - c1) < r1 + 1 - 1e-12:
                        continue
                    dmin = np.min(np.linalg.norm(z - p, axis=1))
                    assert dmin > 1 - 1e-12 and dmin < 1 + (L / 400) ** 2
    # equal unit radii: the unit-disk peanut (perimeter 6 pi - 8 psi)
    ci, ck = np.zeros(2), np.array([2.01, 0.0])
    z = peanut_nodes(ci, ck, 400)
    psi = math.atan2(math.sqrt(4 - 2.01 ** 2 / 4), 2.01 / 2)
    steps = np.linalg.norm(np.diff(np.vstack([z, z[:1]]), axis=0), axis=1)
    assert abs(steps.sum() - (6 * math.pi - 8 * psi)) < 1e-3
