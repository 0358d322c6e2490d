"""Pins of the oracle's flow evaluation and boundary residual (oracle/flow.py).

* P11 single disk: the exterior flow of a disk of radius a under force F and torque t is
  F/(4 pi mu) [-ln r I + r r^T / r^2] + F a^2/(8 pi mu) [I / r^2 - 2 r r^T / r^4]
  + t (x - c)^perp / (4 pi mu r^2) (Stokeslet, potential dipole and rotlet; on r = a it is
  the rigid motion v = F (1/2 - ln a)/(4 pi mu), omega = t/(4 pi mu a^2)).  Resistance
  inverts the same relation.
* P12 near field against brute force: the two-body representation with its fine sources
  reproduces, at fluid points in and around the gap of a pair at gap 1e-3, the flow of a
  direct fine-grid MFS solve of the same problem (no compression, no preconditioning),
  for a pair and for a pair with a third, distant disk.  The compressed coarse form alone
  is far off inside the peanut and equal outside it: the fine term carries the near field.
* P13 boundary residual (eqs. residual_x, residual): below 1e-5 for a mobility pair at gap
  1e-3 with the paper's coarse parameters (the accuracy the paper reports), O(1) without
  the fine correction; of the order of the ring's MFS error for a single disk.
* the peanut membership test: disks, waist, and the rolling circles' exclusion.
"""

import math

import numpy as np
import pytest

from oracle.direct import direct_solve
from oracle.flow import boundary_residual, fine_data, flow_eval, in_peanut
from oracle.geometry import fine_nodes, fine_sources, perp, ring, ring_radius
from oracle.kernel import direct_sum
from oracle.params import MFSParams
from oracle.system import System, solve

PAPER_COARSE = (60, 72, 1 - 12 * math.log(10) / 60)


def _disk_field(x, c, a, F, t, mu=1.0):
    d = x - c
    r2 = np.sum(d * d, axis=1)[:, None]
    dd = np.sum(d * F[None, :], axis=1)[:, None]
    st = (-0.5 * np.log(r2) * F[None, :] + d * dd / r2) / (4 * math.pi * mu)
    dip = a * a * (F[None, :] / r2 - 2 * d * dd / (r2 * r2)) / (8 * math.pi * mu)
    rot = t * perp(d) / r2 / (4 * math.pi * mu)
    return st + dip + rot


@pytest.mark.parametrize("problem", ["mobility", "resistance"])
def test_single_disk_exterior_flow(problem):
    a, mu = 1.3, 1.7
    c = np.array([0.4, -0.2])
    S = System(c[None], a, 36, 72, 0.7, problem, MFSParams(mu=mu))
    if problem == "mobility":
        F, t = np.array([0.8, -0.5]), 1.1
        given = np.array([[F[0], F[1], t]])
    else:
        v, w = np.array([0.3, 0.9]), -0.6
        given = np.array([[v[0], v[1], w]])
        F = v * 4 * math.pi * mu / (0.5 - math.log(a))
        t = w * 4 * math.pi * mu * a * a
    out, mu_sol, _ = solve(S, given, 1e-13)
    ang = np.linspace(0, 2 * math.pi, 7, endpoint=False)
    x = np.concatenate([c + r * np.stack([np.cos(ang + r), np.sin(ang + r)], axis=1) for r in (1.2 * a, 2 * a, 6.0)])
    u = flow_eval(S, mu_sol, x, -np.ones(len(x)), given=given)
    ref = _disk_field(x, c, a, F, t, mu)
    err = np.abs(u - ref).max() / np.abs(ref).max()
    assert err < 1e-8, err
    # on the boundary the flow is the rigid motion up to the MFS error between the
    # collocation nodes, of the order of 0.7^36 = 2.6e-6 for 36 sources on radius 0.7 a
    rigid = out if problem == "mobility" else given
    _, em = boundary_residual(S, mu_sol, rigid, 100, given=given)
    assert em < 1e-5, em


def _fine_ring_body(c, prm):
    Rf = ring_radius(prm.n_fp, prm.eps_ring)
    return (c, ring(c, Rf, prm.n_fp), ring(c, 1.0, int(math.ceil(prm.a_f * prm.n_fp))))


@pytest.mark.parametrize("problem", ["mobility", "resistance"])
def test_near_field_matches_direct_fine_solve(problem):
    prm = MFSParams()
    nc, mc, rc = PAPER_COARSE
    c = np.array([[0.1, 0.2], [0.1 + 2.001 * math.cos(0.7), 0.2 + 2.001 * math.sin(0.7)], [-2.6, 3.6]])
    rng = np.random.default_rng(5)
    e = (c[1] - c[0]) / np.linalg.norm(c[1] - c[0])
    n = perp(e)
    mid = c[0] + 1.0005 * e
    pts = np.array([mid, mid + 0.01 * n, mid - 0.03 * n, mid + 0.1 * n, mid + 0.3 * n,   # in the peanut
                    c[0] - 1.05 * e, c[0] + 3 * n, c[1] + 1.2 * e, mid + 1.2 * n])          # outside
    inside = in_peanut(pts, c[0], c[1], 1.0, 1.0)
    assert inside.tolist() == [True] * 5 + [False] * 4
    for P in (2, 3):
        g = rng.standard_normal((P, 3))
        if problem == "mobility":
            g[:, :2] -= g[:, :2].mean(0)
        S = System(c[:P], 1.0, nc, mc, rc, problem, prm)
        assert len(S.pairs) == 1
        _, mu_sol, _ = solve(S, g, 1e-13)
        Yi, Yk = fine_sources(c[0], c[1], prm)
        Xi, Xk = fine_nodes(c[0], c[1], prm)
        bodies = [(c[0], Yi, Xi), (c[1], Yk, Xk)] + ([_fine_ring_body(c[2], prm)] if P == 3 else [])
        _, Yd, sd = direct_solve(bodies, g, problem, strengths=True)
        ref = direct_sum(pts, Yd, sd.reshape(-1, 2))
        fd = fine_data(S)
        u = flow_eval(S, mu_sol, pts, -np.ones(len(pts)), given=g, fine=fd)
        u0 = flow_eval(S, mu_sol, pts, -np.ones(len(pts)), given=g, use_fine=False)
        scale = np.abs(ref).max()
        err = np.abs(u - ref).max(axis=1) / scale
        err0 = np.abs(u0 - ref).max(axis=1) / scale
        # MFS accuracy of the two discretisations (measured: mobility 1e-6; resistance 2e-10
        # for the pair, 7e-8 with the third disk's coarse ring)
        assert err.max() < (5e-6 if problem == "mobility" else 5e-7), (problem, P, err)
        assert err0[inside].min() > 1e-2                    # the compressed form fails in the peanut
        # same terms in another BLAS order; the compressed strengths are ~10^3 times the field here
        assert np.abs(u0[~inside] - u[~inside]).max() <= 1e-10 * scale


def test_pair_boundary_residual_below_paper_bar():
    prm = MFSParams()
    nc, mc, rc = PAPER_COARSE
    c = np.array([[0.0, 0.0], [2.001, 0.0]])
    g = np.random.default_rng(8).standard_normal((2, 3))
    g[:, :2] -= g[:, :2].mean(0)
    S = System(c, 1.0, nc, mc, rc, "mobility", prm)
    out, mu_sol, _ = solve(S, g, 1e-13)
    fd = fine_data(S)
    eps, em = boundary_residual(S, mu_sol, out, 400, given=g, fine=fd)
    assert eps.shape == (800,)
    assert em < 1e-5, em
    _, em0 = boundary_residual(S, mu_sol, out, 400, given=g, use_fine=False)
    assert em0 > 1.0, em0


def test_peanut_membership():
    ci, ck = np.array([0.0, 0.0]), np.array([2.1, 0.0])
    # rolling unit circle centres at (1.05, +-h), h = sqrt(4 - 1.05^2)
    h = math.sqrt(4 - 1.05 ** 2)
    pts = np.array([[0.3, 0.2], [2.5, -0.5], [1.05, 0.0], [1.05, 0.98 * (h - 1)], [1.05, 1.02 * (h - 1)],
                    [1.05, -1.02 * (h - 1)], [-1.01, 0.0], [1.05, 3.0]])
    assert in_peanut(pts, ci, ck, 1.0, 1.0).tolist() == [True, True, True, True, False, False, False, False]
