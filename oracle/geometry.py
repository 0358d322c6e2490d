"""Point sets of the method (oracle): coarse rings, rigid maps, contacts, fine sets, peanut.

Readings taken here (the paper is silent or ambiguous):

* every equispaced grid (coarse sources, coarse nodes, fine proxies, fine
  equispaced nodes) starts at angle 0 in the global frame; grids do not
  rotate with the pair (Sec. 5, remark on combining fine sources).
* the ellipse focus a is the image accumulation radius R_acc(delta), so the
  segment [0, R_acc] between the foci is shielded (Sec. 5).
* a_ell * N_ell Moebius nodes are added for every contact pair, densest
  toward the neighbour; per disk M_f = ceil(a_f N_fp) + a_ell N_ell.
* the peanut is two convex arcs of the disk boundaries (far sides) and two
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


def limit_point(a1, a2, d):
    """Limit point x_1 (distance from the centre of disk 1 toward disk 2) of the coaxal system of
    two circles of radii a1, a2 at centre distance d: the common fixed point, inside disk 1, of
    the inversions in both circles, where the images of a source accumulate (Sec. 5; the paper
    treats unit disks only, and this point is the reading taken for unequal radii).  For
    a1 = a2 = 1 it is R_acc(d - 2)."""
    b = d * d + a1 * a1 - a2 * a2
    return (b - math.sqrt(b * b - 4.0 * d * d * a1 * a1)) / (2.0 * d)


def fine_count(radius, prm):
    """Fine proxy count of a disk: N_fp scales with the radius (150 at radius 1; a reading of the paper)."""
    return int(round(prm.n_fp * radius))


def ellipse_points(delta, prm, a1=1.0, a2=1.0):
    """Shielding ellipse nodes z(theta_j) in the body-local frame (pair axis = +x), Sec. 5.

    With x1 the limit point of the disk (radius a1) toward its neighbour (radius a2) at gap
    delta: z(theta) = (x1/2)[1 + cos(theta + i alpha)], alpha = arcosh(1 + 2 gamma (a1 - x1)/x1),
    the ellipse with foci 0 and x1 and tip x1 + gamma (a1 - x1); theta_j = (j + 1/2) pi / N_ell,
    j = 0 .. 2 N_ell - 1; keep |z| > R_f (the disk's proxy radius).  Empty when x1 <= R_f.
    For unit disks x1 = R_acc(delta).  Returned as complex numbers.
    """
    Rf = a1 * ring_radius(fine_count(a1, prm), prm.eps_ring)
    x1 = limit_point(a1, a2, a1 + a2 + delta) if (a1, a2) != (1.0, 1.0) else r_acc(delta)
    if x1 <= Rf:
        return np.zeros(0, dtype=np.complex128)
    alpha = math.acosh(1.0 + 2.0 * prm.gamma * (a1 - x1) / x1)
    th = (np.arange(2 * prm.n_ell) + 0.5) * math.pi / prm.n_ell
    z = 0.5 * x1 * (1.0 + np.cos(th + 1j * alpha))
    return z[np.abs(z) > Rf]


def fine_sources(ci, ck, prm, ai=1.0, ak=1.0):
    """Fine source set of the pair (Sec. 5): [proxies_i, ellipse_i], [proxies_k, ellipse_k].

    Proxies: N_fp(a) points on the circle of radius a R_f(N_fp(a)) about each centre (global
    angles).  Ellipse sources: c_i + e^{i phi} z_j (disk i's ellipse) and c_k - e^{i phi} z'_j
    (disk k's, toward i), with e^{i phi} the unit direction from c_i to c_k.  Returns
    (Y_i (n_i,2), Y_k (n_k,2)); for equal radii both have the same length.
    """
    ci, ck, d, e = _pair_frame(ci, ck)
    eu = e[0] + 1j * e[1]
    out = []
    for c0, a0, a1, sgn in ((ci, ai, ak, 1.0), (ck, ak, ai, -1.0)):
        nf = fine_count(a0, prm)
        Rf = a0 * ring_radius(nf, prm.eps_ring)
        ez = sgn * eu * ellipse_points(d - ai - ak, prm, a0, a1)
        out.append(np.concatenate([ring(c0, Rf, nf), c0[None, :] + np.stack([ez.real, ez.imag], axis=1)], axis=0))
    return out[0], out[1]


def fine_nodes(ci, ck, prm, ai=1.0, ak=1.0):
    """Fine collocation nodes of the pair (Sec. 5): per disk ceil(a_f N_fp(a)) equispaced
    nodes plus a_ell N_ell Moebius-mapped nodes theta~ = pi + arg((e^{it} + r)/(1 + r e^{it})),
    t = 2 pi j / M_ell, on the disk's boundary, placed so that theta~ = pi faces the
    neighbour (a reading of the paper).  Returns (X_i, X_k)."""
    ci, ck, d, e = _pair_frame(ci, ck)
    phi = math.atan2(e[1], e[0])
    m_ell = int(prm.a_ell * prm.n_ell)
    t = 2.0 * math.pi * np.arange(m_ell) / m_ell
    w = np.exp(1j * t)
    tt = math.pi + np.angle((w + prm.mobius_r) / (1.0 + prm.mobius_r * w))
    out = []
    for c0, a0, ang in ((ci, ai, phi + tt - math.pi), (ck, ak, phi + tt)):
        m_eq = int(math.ceil(prm.a_f * fine_count(a0, prm) - 1e-12))
        out.append(np.concatenate([ring(c0, a0, m_eq),
                                   c0[None, :] + a0 * np.stack([np.cos(ang), np.sin(ang)], axis=1)], axis=0))
    return out[0], out[1]


def peanut_nodes(ci, ck, m_p, ai=1.0, ak=1.0, rho=1.0):
    """M_p nodes uniform in arc length on the peanut of the pair (Sec. 3.3; unequal radii: a rolling unit circle).

    The peanut is the outline of the two disks with the concave gaps filled by a circle of
    radius rho rolled around the pair (rho = 1, the smallest disk).  With e the unit axis
    from c_i to c_k, n = e^perp and d = |c_k - c_i|, the rolling circle touching both disks
    is centred at c_i + s e +/- h n, s = ((a_i + rho)^2 - (a_k + rho)^2 + d^2) / (2 d),
    h = sqrt((a_i + rho)^2 - s^2); it touches disk i at angle psi_i = atan2(h, s) and disk k
    at pi - psi_k, psi_k = atan2(h, d - s).  Going counter-clockwise from the far point of
    disk i: disk-i arc (pi .. 2 pi - psi_i about c_i), lower concave arc (pi - psi_i down to
    psi_k about the lower rolling centre), disk-k arc (pi + psi_k .. 3 pi - psi_k about c_k),
    upper concave arc (-psi_k down to psi_i - pi about the upper centre), disk-i arc
    (psi_i .. pi).  Angles in the (e, n) frame.  Unit disks: perimeter 6 pi - 8 psi.
    """
    ci, ck, d, e = _pair_frame(ci, ck)
    n = perp(e)
    s = ((ai + rho) ** 2 - (ak + rho) ** 2 + d * d) / (2.0 * d)
    h = math.sqrt((ai + rho) ** 2 - s * s)
    psi_i = math.atan2(h, s)
    psi_k = math.atan2(h, d - s)
    m_lo = ci + s * e - h * n
    m_hi = ci + s * e + h * n
    segs = [  # (centre, radius, start angle, signed sweep)
        (ci, ai, math.pi, math.pi - psi_i),
        (m_lo, rho, math.pi - psi_i, -(math.pi - psi_i - psi_k)),
        (ck, ak, math.pi + psi_k, 2.0 * math.pi - 2.0 * psi_k),
        (m_hi, rho, -psi_k, -(math.pi - psi_i - psi_k)),
        (ci, ai, psi_i, math.pi - psi_i),
    ]
    lengths = np.array([r * abs(sw) for _, r, _, sw in segs])
    total = lengths.sum()
    t = np.arange(m_p) * total / m_p
    out = np.empty((m_p, 2))
    start = np.concatenate([[0.0], np.cumsum(lengths)[:-1]])
    for p in range(m_p):
        j = int(np.searchsorted(start, t[p], side="right") - 1)
        cen, r, a0, sw = segs[j]
        ang = a0 + math.copysign((t[p] - start[j]) / r, sw)
        out[p] = cen + r * (math.cos(ang) * e + math.sin(ang) * n)
    return out
