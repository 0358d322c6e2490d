"""Pins of the oracle's Stokeslet and direct sum (eq. stokeslet2d, eq. stokes_sum)."""

import math

import numpy as np

from oracle.kernel import direct_sum, stokeslet_blocks, stokeslet_matrix


def _u(x, y, f, mu=1.0):
    return stokeslet_blocks(np.atleast_2d(x), np.atleast_2d(y), mu)[0, 0] @ f


def test_symmetry():
    # S(x, y) = S(y, x) = S(x, y)^T
    rng = np.random.default_rng(0)
    x = rng.standard_normal((7, 2))
    y = rng.standard_normal((5, 2)) + 3.0
    a = stokeslet_blocks(x, y)
    b = stokeslet_blocks(y, x)
    assert np.allclose(a, b.transpose(1, 0, 2, 3), rtol=0, atol=1e-15)
    assert np.allclose(a, a.transpose(0, 1, 3, 2), rtol=0, atol=1e-15)


def test_divergence_free():
    # div_x S(x, y) f = 0: centred differences, h = 1e-4 -> O(h^2) truncation.
    # Pins the relative weight and sign of the log and dyadic terms.
    rng = np.random.default_rng(1)
    h = 1e-4
    for _ in range(20):
        y = rng.standard_normal(2)
        x = y + rng.uniform(0.3, 3.0) * np.array([math.cos(t := rng.uniform(0, 6.3)), math.sin(t)])
        f = rng.standard_normal(2)
        dux = (_u(x + [h, 0], y, f) - _u(x - [h, 0], y, f))[0] / (2 * h)
        duy = (_u(x + [0, h], y, f) - _u(x - [0, h], y, f))[1] / (2 * h)
        scale = np.linalg.norm(f) / np.linalg.norm(x - y)
        assert abs(dux + duy) < 1e-7 * scale


def test_zero_net_flux_through_circle():
    # Incompressibility in integral form: the flux of a Stokeslet field through a
    # circle enclosing the source vanishes (trapezoid rule, spectrally accurate).
    y = np.array([0.2, -0.1])
    f = np.array([0.7, -1.3])
    n = 256
    t = 2 * math.pi * np.arange(n) / n
    nrm = np.stack([np.cos(t), np.sin(t)], axis=1)
    pts = 1.5 * nrm
    u = direct_sum(pts, y[None], f[None])
    flux = np.sum(np.sum(u * nrm, axis=1)) * (2 * math.pi * 1.5 / n)
    assert abs(flux) < 1e-13


def test_ring_of_tangential_forces_is_a_rotlet():
    # N equal tangential point forces on a ring of radius rho with total torque t:
    # outside the ring the flow is the rotlet t/(4 pi mu) (x-c)^perp / |x-c|^2 up to
    # O((rho/r)^N) (rotating-cylinder flow).  Pins the 1/(4 pi mu) normalisation and sign.
    for mu in (1.0, 2.5):
        N, rho, t = 64, 0.5, 1.7
        th = 2 * math.pi * np.arange(N) / N
        y = rho * np.stack([np.cos(th), np.sin(th)], axis=1)
        lam = (t / (N * rho)) * np.stack([-np.sin(th), np.cos(th)], axis=1)
        x = np.array([[2.0, 0.3], [-1.1, 1.9], [0.0, -3.0]])
        u = direct_sum(x, y, lam, mu)
        r2 = np.sum(x * x, axis=1)
        ref = t / (4 * math.pi * mu) * np.stack([-x[:, 1], x[:, 0]], axis=1) / r2[:, None]
        assert np.max(np.abs(u - ref)) < 1e-14 * 1e3


def test_direct_sum_equals_matrix_and_parallel_split():
    rng = np.random.default_rng(2)
    x = rng.uniform(-5, 5, (300, 2))
    y = rng.uniform(-5, 5, (211, 2)) + 0.001
    s = rng.standard_normal((211, 2))
    u1 = direct_sum(x, y, s)
    u2 = (stokeslet_matrix(x, y) @ s.reshape(-1)).reshape(-1, 2)
    u3 = direct_sum(x, y, s, workers=3, chunk_elems=5000)
    assert np.allclose(u1, u2, rtol=1e-13, atol=1e-13)
    assert np.allclose(u1, u3, rtol=1e-14, atol=1e-14)
