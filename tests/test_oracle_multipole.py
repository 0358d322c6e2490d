"""Pins of the far-field expansion of a ring of Stokeslets (oracle/multipole.py).

* against the direct Stokeslet sum (oracle/kernel.py, eq. stokeslet2d) for random
  strengths on rings of several sizes and radii, at theta = rho/|Z| = 1/4 and 1/2:
  the truncated expansion stays below sum |sigma| theta^(p+1) / (1 - theta) / (4 pi mu);
* the error falls geometrically with the order p (ratio ~theta), and at high order the
  expansion equals the direct sum to rounding;
* the special strengths of the mobility problem (zero net force and torque after the
  rigid projection): S0 = 0 and B_1 real, and the expansion still matches.
"""

import math

import numpy as np
import pytest

from oracle.geometry import rigid_map, rigid_projector, ring
from oracle.kernel import direct_sum
from oracle.multipole import cluster_moments, eval_local, far_field, far_field_general, local_expansion, moments


def _case(n, rho, seed, project=False):
    rng = np.random.default_rng(seed)
    c = np.array([0.3, -0.4])
    y = ring(c, rho, n)
    sig = rng.standard_normal((n, 2))
    if project:
        K = rigid_map(y, c)
        sig = (sig.reshape(-1) - rigid_projector(K) @ sig.reshape(-1)).reshape(-1, 2)
    w = (y[:, 0] - c[0]) + 1j * (y[:, 1] - c[1])
    s = sig[:, 0] + 1j * sig[:, 1]
    return c, y, sig, w, s


def _points(c, R, m=11):
    ang = np.linspace(0, 2 * math.pi, m, endpoint=False) + 0.3
    return c + R * np.stack([np.cos(ang), np.sin(ang)], axis=1)


@pytest.mark.parametrize("n,rho", [(36, 0.7), (50, 0.98), (7, 0.5)])
def test_truncated_expansion_within_bound(n, rho):
    mu = 1.3
    c, y, sig, w, s = _case(n, rho, 1)
    for theta in (0.25, 0.5):
        x = _points(c, rho / theta)
        ref = direct_sum(x, y, sig, mu)
        Z = (x[:, 0] - c[0]) + 1j * (x[:, 1] - c[1])
        for p in (4, 8, 12):
            A, B = moments(w, s, p)
            u = far_field(Z, A, B, rho, mu)
            err = np.abs(np.stack([u.real, u.imag], axis=1) - ref).max()
            bound = np.abs(s).sum() * theta ** (p + 1) / (1 - theta) / (4 * math.pi * mu)
            assert err <= bound, (n, rho, theta, p, err, bound)


def test_error_falls_geometrically_and_high_order_is_exact():
    c, y, sig, w, s = _case(36, 0.7, 2)
    theta = 0.5
    x = _points(c, 0.7 / theta)
    ref = direct_sum(x, y, sig)
    Z = (x[:, 0] - c[0]) + 1j * (x[:, 1] - c[1])
    errs = []
    for p in (6, 12, 18):
        u = far_field(Z, *moments(w, s, p), 0.7)
        errs.append(np.abs(np.stack([u.real, u.imag], axis=1) - ref).max())
    assert errs[1] < 0.5 ** 5 * errs[0] and errs[2] < 0.5 ** 5 * errs[1]
    x = _points(c, 0.7 / 0.25)                      # theta = 1/4, p = 30: truncation 1e-19
    ref = direct_sum(x, y, sig)
    Z = (x[:, 0] - c[0]) + 1j * (x[:, 1] - c[1])
    u = far_field(Z, *moments(w, s, 30), 0.7)
    assert np.abs(np.stack([u.real, u.imag], axis=1) - ref).max() < 1e-13 * np.abs(ref).max()


def test_mobility_strengths_zero_force_and_torque():
    c, y, sig, w, s = _case(36, 0.7, 3, project=True)
    A, B = moments(w, s, 12)
    assert abs(A[0]) < 1e-13 and abs(B[1].imag) < 1e-13   # net force, torque = Im(sum conj(w) sigma)
    x = _points(c, 0.7 / 0.25)
    ref = direct_sum(x, y, sig)
    Z = (x[:, 0] - c[0]) + 1j * (x[:, 1] - c[1])
    u = far_field(Z, A, B, 0.7)
    bound = np.abs(s).sum() * 0.25 ** 13 / 0.75 / (4 * math.pi)
    assert np.abs(np.stack([u.real, u.imag], axis=1) - ref).max() <= bound


def _cluster(seed, n_disks=9, spread=2.5):
    # sources of several rings scattered around the origin: a cluster of disks
    rng = np.random.default_rng(seed)
    cs = rng.uniform(-spread, spread, (n_disks, 2))
    y = np.concatenate([ring(cc, 0.7, 36) for cc in cs])
    sig = rng.standard_normal(y.shape)
    return y, sig


@pytest.mark.parametrize("seed", [4, 5])
def test_cluster_expansion_within_bound(seed):
    mu = 0.8
    y, sig = _cluster(seed)
    C = np.array([0.2, -0.1])
    w = (y[:, 0] - C[0]) + 1j * (y[:, 1] - C[1])
    s = sig[:, 0] + 1j * sig[:, 1]
    Rc = np.abs(w).max()
    for theta in (0.25, 0.5):
        x = _points(C, Rc / theta, 13)
        ref = direct_sum(x, y, sig, mu)
        Z = (x[:, 0] - C[0]) + 1j * (x[:, 1] - C[1])
        for p in (6, 12):
            u = far_field_general(Z, *cluster_moments(w, s, p), mu)
            err = np.abs(np.stack([u.real, u.imag], axis=1) - ref).max()
            bound = np.abs(s).sum() * theta ** (p + 1) / (1 - theta) / (4 * math.pi * mu)
            assert err <= bound, (theta, p, err, bound)
    x = _points(C, Rc / 0.25, 7)                     # p = 30: the direct sum to rounding
    ref = direct_sum(x, y, sig)
    Z = (x[:, 0] - C[0]) + 1j * (x[:, 1] - C[1])
    u = far_field_general(Z, *cluster_moments(w, s, 30))
    assert np.abs(np.stack([u.real, u.imag], axis=1) - ref).max() < 1e-13 * np.abs(ref).max()


def test_cluster_moments_of_a_ring_reduce_to_the_ring_form():
    c, y, sig, w, s = _case(36, 0.7, 6)
    A, B, D = cluster_moments(w, s, 10)
    assert abs(D[0] - B[1]) < 1e-13 * np.abs(s).sum()
    assert np.allclose(D[1:], 0.49 * A[:-1], rtol=0, atol=1e-13 * np.abs(s).sum())
    # the two truncations differ by one term of Q; at order 30 both are the full series
    A, B, D = cluster_moments(w, s, 30)
    x = _points(c, 0.7 / 0.3)
    Z = (x[:, 0] - c[0]) + 1j * (x[:, 1] - c[1])
    assert np.allclose(far_field_general(Z, A, B, D), far_field(Z, A, B, 0.7), rtol=0, atol=1e-15)


def _local_sum(groups, T, q, p):
    """Sum of the local expansions about T of several source groups (sources y, strengths sig,
    expansion centre C): (L1, L2, const)."""
    L1 = np.zeros(q + 1, complex)
    L2 = np.zeros(q + 1, complex)
    const = 0.0
    for y, sig, C in groups:
        w = (y[:, 0] - C[0]) + 1j * (y[:, 1] - C[1])
        s = sig[:, 0] + 1j * sig[:, 1]
        a, b, cst = local_expansion(*cluster_moments(w, s, p), complex(T[0] - C[0], T[1] - C[1]), q)
        L1, L2, const = L1 + a, L2 + b, const + cst
    return L1, L2, const


@pytest.mark.parametrize("direction", [(1.0, 0.6), (-1.0, 1e-9), (-1.0, -1e-9), (-0.3, -1.0)])
def test_local_expansion_matches_direct_sum(direction):
    # two clusters of rings (radius Rc about their centres) and targets within rt of T; the
    # directions include Delta = T - C just above and below the negative real axis, where a
    # complex log would jump by 2 pi i
    mu = 1.1
    y1, s1 = _cluster(7)
    y2, s2 = _cluster(8)
    d = np.array(direction) / np.linalg.norm(direction)
    C1, C2 = np.array([0.0, 0.0]), -9.0 * d + 3.0 * np.array([-d[1], d[0]])
    y2 = y2 + C2
    Rc = max(np.abs(y1 - C1).max(), np.abs(y2 - C2).max()) * math.sqrt(2)
    rt = 2.0
    T = C1 + d * 3.2 * (Rc + rt)
    rng = np.random.default_rng(9)
    x = T + rng.uniform(-1, 1, (40, 2)) * rt / math.sqrt(2)
    ref = direct_sum(x, np.concatenate([y1, y2]), np.concatenate([s1, s2]), mu)
    theta = max((Rc + rt) / np.linalg.norm(T - C) for C in (C1, C2))
    assert theta < 0.35
    sabs = np.abs(np.concatenate([s1, s2])).sum(1).sum()
    wt = (x[:, 0] - T[0]) + 1j * (x[:, 1] - T[1])
    errs = []
    for p in (10, 20, 30):
        u = eval_local(wt, *_local_sum([(y1, s1, C1), (y2, s2, C2)], T, p, p), mu)
        err = np.abs(np.stack([u.real, u.imag], axis=1) - ref).max()
        errs.append(err)
        assert err <= 10 * sabs * theta ** (p + 1) / (1 - theta) / (4 * math.pi * mu), (p, err)
    assert errs[2] < 1e-13 * np.abs(ref).max()


def test_local_expansion_of_mobility_strengths():
    # zero net force and torque per disk (the mobility matvec's strengths): the field decays
    # faster, and the expansion keeps the error relative to it
    rng = np.random.default_rng(10)
    cs = rng.uniform(-2.5, 2.5, (9, 2))
    ys, ss = [], []
    for cc in cs:
        y = ring(cc, 0.7, 36)
        K = rigid_map(y, cc)
        sg = rng.standard_normal(72)
        ys.append(y)
        ss.append((sg - rigid_projector(K) @ sg).reshape(-1, 2))
    y, sig = np.concatenate(ys), np.concatenate(ss)
    C = np.zeros(2)
    T = np.array([-14.0, 10.0])
    x = T + rng.uniform(-1, 1, (30, 2))
    ref = direct_sum(x, y, sig)
    u = eval_local((x[:, 0] - T[0]) + 1j * (x[:, 1] - T[1]), *_local_sum([(y, sig, C)], T, 26, 26))
    assert np.abs(np.stack([u.real, u.imag], axis=1) - ref).max() < 1e-12 * np.abs(ref).max()
