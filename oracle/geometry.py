"""Point sets of the method (oracle): coarse rings, rigid maps, contacts, fine sets, peanut.

Readings taken here (the paper is silent or ambiguous):

* Q3  every equispaced grid (coarse sources, coarse nodes, fine proxies, fine
      equispaced nodes) starts at angle 0 in the global frame; grids do not
      rotate with the pair (Sec. 5, remark on combining fine sources).
* Q13 the ellipse focus a is the image accumulation radius R_acc(delta), so the
      segment [0, R_acc] between the foci is shielded (Sec. 5).
* Q15 a_ell * N_ell Moebius nodes are added for every contact pair, densest
      toward the neighbour; per disk M_f = ceil(a_f N_fp) + a_ell N_ell.
* Q16 the peanut is two convex arcs of the disk boundaries (far sides) and two
      concave arcs of the unit circle rolled around the pair; M_p nodes uniform
      in arc length starting at the far point of body i, counter-clockwise.
"""

from __future__ import annotations

import math

import numpy as np


def perp(v):
    """(v1, v2)^perp = (-v2, v1) (Sec. 1, after eq. rigidbc)."""
    v = np.asarray(v, dtype=np.float64)
    return np.stack([-v[..., 1], v[..., 0]], axis=-1)


def ring(center, radius, n):
    """n points equispaced on the circle |p - center| = radius, first at angle 0."""
    t = 2.0 * math.pi * np.arange(n) / n
    return np.asarray(center, dtype=np.float64)[None, :] + radius * np.stack([np.cos(t), np.sin(t)], axis=1)


def ring_radius(n, eps):
    """R = 1 - ln(1/eps)/N (Sec. 6, rule for the coarse and fine proxy radii)."""
    return 1.0 - math.log(1.0 / eps) / n


def rigid_map(points, center):
    """eq. Kmat: rows [I_2, (p - c)^perp] for each point; shape (2n, 3).

    K^T lambda gives (force_x, force_y, torque) of strengths lambda at the points;
    the same construction at boundary nodes gives B, mapping (v, omega) to the
    rigid velocity v + omega (x - c)^perp of eq. rigidbc.
    """
    p = np.asarray(points, dtype=np.float64).reshape(-1, 2) - np.asarray(center, dtype=np.float64)[None, :]
    n = p.shape[0]
    K = np.zeros((2 * n, 3))
    K[0::2, 0] = 1.0
    K[1::2, 1] = 1.0
    K[0::2, 2] = -p[:, 1]
    K[1::2, 2] = p[:, 0]
    return K


def rigid_projector(K):
    """L = K (K^T K)^{-1} K^T, the projector onto rigid-body strengths (Sec. 4.1)."""
    return K @ np.linalg.solve(K.T @ K, K.T)


def r_acc(delta):
    """Image accumulation radius R_acc(delta) = 1 + delta/2 - sqrt(delta + delta^2/4) (Sec. 5)."""
    return 1.0 + 0.5 * delta - math.sqrt(delta + 0.25 * delta * delta)


def contacts(centers, radii, delta_c):
    """All pairs i < k with |c_i - c_k| <= a_i + a_k + delta_c (Sec. 6; Alg. 2 precompute), brute force."""
    c = np.asarray(centers, dtype=np.float64)
    a = np.asarray(radii, dtype=np.float64)
    P = c.shape[0]
    out = []
    blk = 2048
    for lo in range(0, P, blk):
        hi = min(P, lo + blk)
        d = np.sqrt(((c[lo:hi, None, :] - c[None, :, :]) ** 2).sum(-1))
        lim = a[lo:hi, None] + a[None, :] + delta_c
        ii, kk = np.nonzero(d <= lim)
        gi = ii + lo
        sel = kk > gi
        out.append(np.stack([gi[sel], kk[sel]], axis=1))
    pr = np.concatenate(out, axis=0) if out else np.zeros((0, 2), dtype=np.int64)
    order = np.lexsort((pr[:, 1], pr[:, 0]))
    return pr[order].astype(np.int64)


def _pair_frame(ci, ck):
    ci = np.asarray(ci, dtype=np.float64)
    ck = np.asarray(ck, dtype=np.float64)
    dv = ck - ci
    d = math.hypot(dv[0], dv[1])
    return ci, ck, d, dv / d


def ellipse_points(delta, prm):
    """Shielding ellipse nodes z(theta_j) in the body-local frame (pair axis = +x), Sec. 5.

    z(theta) = (a/2)[1 + cos(theta + i alpha)], alpha = arcosh(1 + 2 gamma (1-a)/a),
    theta_j = (j + 1/2) pi / N_ell, j = 0 .. 2 N_ell - 1; keep |z| > R_f.  Empty
    when R_acc(delta) <= R_f.  Returned as complex numbers.
    """
    Rf = ring_radius(prm.n_fp, prm.eps_ring)
    a = r_acc(delta)
    if a <= Rf:
        return np.zeros(0, dtype=np.complex128)
    alpha = math.acosh(1.0 + 2.0 * prm.gamma * (1.0 - a) / a)
    th = (np.arange(2 * prm.n_ell) + 0.5) * math.pi / prm.n_ell
    z = 0.5 * a * (1.0 + np.cos(th + 1j * alpha))
    return z[np.abs(z) > Rf]


def fine_sources(ci, ck, prm):
    """Fine source set of the pair (Sec. 5): [proxies_i, ellipse_i, proxies_k, ellipse_k].

    Proxies: N_fp points on the circle of radius R_f about each centre (global
    angles).  Ellipse sources: c_i + e^{i phi} z_j and c_k - e^{i phi} z_j with
    e^{i phi} the unit direction from c_i to c_k.  Returns (Y_i (n_i,2), Y_k (n_k,2)).
    """
    ci, ck, d, e = _pair_frame(ci, ck)
    Rf = ring_radius(prm.n_fp, prm.eps_ring)
    z = ellipse_points(d - 2.0, prm)
    ez = (e[0] + 1j * e[1]) * z
    enh = np.stack([ez.real, ez.imag], axis=1)
    Yi = np.concatenate([ring(ci, Rf, prm.n_fp), ci[None, :] + enh], axis=0)
    Yk = np.concatenate([ring(ck, Rf, prm.n_fp), ck[None, :] - enh], axis=0)
    return Yi, Yk


def fine_nodes(ci, ck, prm):
    """Fine collocation nodes of the pair (Sec. 5): per disk ceil(a_f N_fp) equispaced
    nodes plus a_ell N_ell Moebius-mapped nodes theta~ = pi + arg((e^{it} + r)/(1 + r e^{it})),
    t = 2 pi j / M_ell, placed so that theta~ = pi faces the neighbour (Q15).
    Returns (X_i, X_k), each (M_f, 2)."""
    ci, ck, d, e = _pair_frame(ci, ck)
    phi = math.atan2(e[1], e[0])
    m_eq = int(math.ceil(prm.a_f * prm.n_fp - 1e-12))
    m_ell = int(prm.a_ell * prm.n_ell)
    t = 2.0 * math.pi * np.arange(m_ell) / m_ell
    w = np.exp(1j * t)
    tt = math.pi + np.angle((w + prm.mobius_r) / (1.0 + prm.mobius_r * w))
    ang_i = phi + tt - math.pi
    ang_k = phi + tt
    Xi = np.concatenate([ring(ci, 1.0, m_eq), ci[None, :] + np.stack([np.cos(ang_i), np.sin(ang_i)], axis=1)], axis=0)
    Xk = np.concatenate([ring(ck, 1.0, m_eq), ck[None, :] + np.stack([np.cos(ang_k), np.sin(ang_k)], axis=1)], axis=0)
    return Xi, Xk


def peanut_nodes(ci, ck, m_p):
    """M_p nodes uniform in arc length on the peanut of two unit disks (Sec. 3.3, Q16).

    With e the unit axis from c_i to c_k, n = e^perp, d = |c_k - c_i| and
    h = sqrt(4 - (d/2)^2), the rolling unit circle touching both disks is centred
    at m +/- h n (m the midpoint).  psi = atan2(h, d/2).  Going counter-clockwise
    from the far point of disk i: disk-i arc (angles pi .. 2 pi - psi about c_i),
    lower concave arc (angles pi - psi down to psi about m - h n), disk-k arc
    (angles pi + psi .. 3 pi - psi about c_k), upper concave arc (angles -psi down
    to psi - pi about m + h n), and disk-i arc (psi .. pi).  Angles are measured in
    the (e, n) frame.  Perimeter 6 pi - 8 psi.
    """
    ci, ck, d, e = _pair_frame(ci, ck)
    n = perp(e)
    h = math.sqrt(4.0 - 0.25 * d * d)
    psi = math.atan2(h, 0.5 * d)
    m = 0.5 * (ci + ck)
    segs = [  # (centre, start angle, signed sweep)
        (ci, math.pi, math.pi - psi),
        (m - h * n, math.pi - psi, -(math.pi - 2.0 * psi)),
        (ck, math.pi + psi, 2.0 * math.pi - 2.0 * psi),
        (m + h * n, -psi, -(math.pi - 2.0 * psi)),
        (ci, psi, math.pi - psi),
    ]
    lengths = np.array([abs(s[2]) for s in segs])
    total = lengths.sum()
    s = np.arange(m_p) * total / m_p
    out = np.empty((m_p, 2))
    start = np.concatenate([[0.0], np.cumsum(lengths)[:-1]])
    for p in range(m_p):
        j = int(np.searchsorted(start, s[p], side="right") - 1)
        cen, a0, sw = segs[j]
        ang = a0 + math.copysign(s[p] - start[j], sw)
        out[p] = cen + math.cos(ang) * e + math.sin(ang) * n
    return out
