"""Flow evaluation with the two-body representation, and the boundary residual (oracle).

Test infrastructure: a plain FP64 CPU reference for the library's flow evaluation; only
tests, the smoke check and the benchmark's CPU baseline use it.

After a solve, the flow at a point x outside the bodies is the two-body representation
(Sec. 3.3, eq. chi; the source triplet that Alg. 2 returns when flowEval is set):

  u(x) = sum_j S(x, Y^(j)) Pi_j lambda_bar^(j)             one-body fields (eq. b1rep)
       + sum_c eta^c(x)                                     pair corrections
       [+ u_0(x) = sum_j S(x, Y^(j)) lambda_0^(j)]          mobility: the force/torque sources

  eta^c(x) = -S(x, Yf^c) Pi_f beta^c,   beta^c = G^c [lambda_bar^(i); lambda_bar^(k)],

G^c = F^+ X the fine map of eq. bfm in the pair's symmetric form (the fine field of beta
reproduces each disk's neighbour's one-body field on it; the correction cancels that
field), Pi_f the per-disk fine projection I - L_f for mobility (Sec. 4.3) and the identity
for resistance.  Outside the peanut of c, eta^c equals the field of the compressed coarse
strengths S(x, Y^c) Pi lambda_tilde^c to the compression accuracy (Sec. 3.3, eq. Amat),
which is what Alg. 3 uses; on the pair's own disks and inside its peanut only the fine
form is accurate.  So each pair contributes its fine field at the points it is near to
(the points of its two disks' boundaries, and fluid points inside its peanut) and its
compressed field everywhere else.

Boundary residual (Sec. 6.1, eqs. residual_x and residual): at boundary points x of body
i, eps(x) = |u(x) - g^(i)(x)| with g^(i)(x) = v_i + omega_i (x - c_i)^perp the rigid motion
(mobility: the solve's velocities; resistance: the prescribed ones), and
eps_max = max_x eps(x) / max_x |g(x)|.
"""

from __future__ import annotations

import math

import numpy as np

from .geometry import fine_sources, perp, rigid_map, rigid_projector
from .kernel import direct_sum, stokeslet_matrix
from .pairs import pair_matrices


def fine_data(S):
    """Per pair: fine sources (Yf_i, Yf_k) and the fine map G (reads the pair matrices again
    with keep=True; the solve itself needs only A and E)."""
    out = []
    for i, k in S.pairs:
        d = pair_matrices(S.c[i], S.c[k], S.cls[i], S.prm, keep=True, ob_k=S.cls[k])
        out.append(dict(Yfi=d["Yfi"], Yfk=d["Yfk"], G=d["G"]))
    return out


def in_peanut(pts, ci, ck, ai, ak, rho=1.0):
    """True for points inside the peanut of the pair (the two disks with the concave gaps filled
    up to a circle of radius rho rolled around the pair; see geometry.peanut_nodes)."""
    pts = np.atleast_2d(pts)
    ci = np.asarray(ci, dtype=np.float64)
    ck = np.asarray(ck, dtype=np.float64)
    d = float(np.linalg.norm(ck - ci))
    e = (ck - ci) / d
    n = perp(e)
    s = ((ai + rho) ** 2 - (ak + rho) ** 2 + d * d) / (2.0 * d)
    h = math.sqrt((ai + rho) ** 2 - s * s)
    m_lo = ci + s * e - h * n
    m_hi = ci + s * e + h * n
    inside = (np.linalg.norm(pts - ci, axis=1) <= ai) | (np.linalg.norm(pts - ck, axis=1) <= ak)
    # the waist: inside the quadrilateral c_i, m_lo, c_k, m_hi (the rolling circles touch the disks
    # on its edges) and outside both rolling circles
    quad = np.array([ci, m_lo, ck, m_hi])
    in_quad = np.ones(pts.shape[0], dtype=bool)
    for q in range(4):
        a, b = quad[q], quad[(q + 1) % 4]
        cross = (b[0] - a[0]) * (pts[:, 1] - a[1]) - (b[1] - a[1]) * (pts[:, 0] - a[0])
        in_quad &= cross >= 0.0
    waist = in_quad & (np.linalg.norm(pts - m_lo, axis=1) >= rho) & (np.linalg.norm(pts - m_hi, axis=1) >= rho)
    return inside | waist


def flow_eval(S, mu, pts, body, given=None, fine=None, use_fine=True):
    """Velocity (n, 2) at points pts (n, 2) from the solution mu of system S.

    body[t] is the body whose boundary holds point t, or -1 for a point in the fluid.
    given: (P, 3) forces/torques for mobility (the u_0 sources), ignored for resistance.
    fine: fine_data(S) (computed here if None).  use_fine=False keeps the compressed form
    for every pair (the representation Alg. 3 evaluates at the coarse nodes of other
    bodies), to show what the fine correction adds.
    """
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 2)
    body = np.asarray(body, dtype=np.int64).reshape(-1)
    mu_v = S.prm.mu
    lam_bar, _, ltil = S.step1(mu)
    # one-body fields (and the mobility force/torque sources)
    sig = S.sigma(lam_bar)
    if S.problem == "mobility":
        given = np.asarray(given, dtype=np.float64).reshape(S.P, 3)
        sig = sig + np.concatenate([ob.K @ np.linalg.solve(ob.K.T @ ob.K, given[i]) for i, ob in enumerate(S.cls)])
    u = direct_sum(pts, S.Y, sig.reshape(-1, 2), mu_v).reshape(-1, 2)
    if use_fine and fine is None and len(S.pairs):
        fine = fine_data(S)
    for c, (i, k) in enumerate(S.pairs):
        ni = 2 * S.n_src[i]
        near = (body == i) | (body == k)
        fluid = body < 0
        if fluid.any():
            near[fluid] = in_peanut(pts[fluid], S.c[i], S.c[k], S.a[i], S.a[k])
        if not use_fine:
            near[:] = False
        far = ~near
        if far.any():   # compressed coarse strengths
            u[far] += (stokeslet_matrix(pts[far], S.Yb(i), mu_v) @ S.cls[i].project(ltil[c][:ni])).reshape(-1, 2)
            u[far] += (stokeslet_matrix(pts[far], S.Yb(k), mu_v) @ S.cls[k].project(ltil[c][ni:])).reshape(-1, 2)
        if near.any():  # fine correction sources
            fd = fine[c]
            x = np.concatenate([S.src_of(lam_bar, i), S.src_of(lam_bar, k)])
            beta = fd["G"] @ x
            nfi = 2 * fd["Yfi"].shape[0]
            bi, bk = beta[:nfi], beta[nfi:]
            if S.problem == "mobility":
                Ki = rigid_map(fd["Yfi"], S.c[i])
                Kk = rigid_map(fd["Yfk"], S.c[k])
                bi = bi - rigid_projector(Ki) @ bi
                bk = bk - rigid_projector(Kk) @ bk
            u[near] -= (stokeslet_matrix(pts[near], fd["Yfi"], mu_v) @ bi).reshape(-1, 2)
            u[near] -= (stokeslet_matrix(pts[near], fd["Yfk"], mu_v) @ bk).reshape(-1, 2)
    return u


def boundary_nodes(S, n_per_body):
    """n_per_body points on each body's boundary at angles 2 pi (j + 1/2) / n (global angles);
    returns points (P n, 2) and their bodies."""
    j = (np.arange(n_per_body) + 0.5) * (2.0 * math.pi / n_per_body)
    ring = np.stack([np.cos(j), np.sin(j)], axis=1)
    pts = np.concatenate([S.c[i] + S.a[i] * ring for i in range(S.P)])
    return pts, np.repeat(np.arange(S.P), n_per_body)


def boundary_residual(S, mu, rigid, n_per_body, given=None, fine=None, use_fine=True):
    """Pointwise residual eps(x) at the boundary nodes and eps_max (eqs. residual_x, residual).

    rigid: (P, 3) rigid motions [v; omega] the boundary velocity should equal (mobility: the
    solve's output; resistance: the prescribed velocities).  given: mobility forces/torques.
    """
    pts, body = boundary_nodes(S, n_per_body)
    u = flow_eval(S, mu, pts, body, given=given, fine=fine, use_fine=use_fine)
    rigid = np.asarray(rigid, dtype=np.float64).reshape(S.P, 3)
    g = rigid[body, :2] + rigid[body, 2:3] * perp(pts - S.c[body])
    eps = np.linalg.norm(u - g, axis=1)
    return eps, float(eps.max() / np.linalg.norm(g, axis=1).max())
