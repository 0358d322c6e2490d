"""Seeded disk packings with the shapes of the paper's workloads.

The paper's large experiments use random packings of unit disks at a prescribed
area fraction and minimum separation (Sec. 6.2), and small clusters in which
every disk is close to a neighbour (Sec. 6.1).  The packings here follow the
benchmark recipes instead: a jittered square grid (16 disks), and a triangular
lattice in a square box that is perturbed, relaxed by pairwise repulsion until
every gap is at least ``g_min``, and finished by moving the closest pair to a
gap of exactly ``g_min``.

Only geometry is produced here (centres, radii, box side).  Nothing in this file
evaluates a Stokeslet or discretises a disk.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.spatial import cKDTree

CONFIG_SEED_BASE = 260611273


def _rng(seed):
    return np.random.default_rng(seed)


def _pairs_within(c, rmax):
    tree = cKDTree(c)
    pr = tree.query_pairs(r=rmax, output_type="ndarray")
    if pr.size == 0:
        return np.zeros((0, 2), dtype=np.int64)
    return pr.astype(np.int64)


def _gaps(c, radii, pr):
    d = np.linalg.norm(c[pr[:, 1]] - c[pr[:, 0]], axis=1)
    return d - radii[pr[:, 0]] - radii[pr[:, 1]], d


def min_gap(c, radii):
    """Smallest surface-to-surface gap over all disk pairs (brute force on a KD tree)."""
    c = np.asarray(c, dtype=np.float64)
    radii = np.broadcast_to(np.asarray(radii, dtype=np.float64), (c.shape[0],))
    if c.shape[0] < 2:
        return np.inf
    rmax = 2.0 * radii.max() + 1.0
    pr = _pairs_within(c, rmax)
    while pr.shape[0] == 0:
        rmax *= 2.0
        pr = _pairs_within(c, rmax)
    g, _ = _gaps(c, radii, pr)
    return float(g.min())


def close_pairs_count(c, radii, delta_c):
    """Number of pairs with gap <= delta_c."""
    c = np.asarray(c, dtype=np.float64)
    radii = np.broadcast_to(np.asarray(radii, dtype=np.float64), (c.shape[0],))
    pr = _pairs_within(c, 2.0 * radii.max() + delta_c)
    if pr.shape[0] == 0:
        return 0
    g, _ = _gaps(c, radii, pr)
    return int(np.count_nonzero(g <= delta_c))


def _relax(c, radii, box, g_target, max_sweeps=4000):
    """Push apart every pair closer than g_target; keep disks inside the box."""
    amax = radii.max()
    for _ in range(max_sweeps):
        pr = _pairs_within(c, 2.0 * amax + g_target)
        if pr.shape[0] == 0:
            return c
        g, d = _gaps(c, radii, pr)
        bad = g < g_target
        if not np.any(bad):
            return c
        pr = pr[bad]
        g = g[bad]
        d = d[bad]
        u = (c[pr[:, 1]] - c[pr[:, 0]]) / d[:, None]
        push = 0.5 * (g_target - g) * 1.05 + 1e-9
        disp = np.zeros_like(c)
        np.add.at(disp, pr[:, 0], -push[:, None] * u)
        np.add.at(disp, pr[:, 1], push[:, None] * u)
        c = c + disp
        if box is not None:
            lo = radii[:, None]
            hi = box - radii[:, None]
            c = np.minimum(np.maximum(c, lo), hi)
    raise RuntimeError("packing relaxation did not converge; lower the area fraction or perturbation")


def _set_closest_gap(c, radii, g_min):
    """Move the closest pair symmetrically along its centre line to gap exactly g_min."""
    amax = radii.max()
    pr = _pairs_within(c, 2.0 * amax + 4.0 * g_min + 0.5)
    g, d = _gaps(c, radii, pr)
    order = np.argsort(g)
    for idx in order[:64]:
        i, k = pr[idx]
        shift = 0.5 * (g[idx] - g_min)
        u = (c[k] - c[i]) / d[idx]
        trial = c.copy()
        trial[i] = c[i] + shift * u
        trial[k] = c[k] - shift * u
        # exact gap by construction; check nobody else got closer than g_min
        gi = np.linalg.norm(trial - trial[i], axis=1) - radii - radii[i]
        gk = np.linalg.norm(trial - trial[k], axis=1) - radii - radii[k]
        gi[i] = np.inf
        gi[k] = np.inf
        gk[i] = np.inf
        gk[k] = np.inf
        if gi.min() >= g_min and gk.min() >= g_min:
            # recompute along the final centre line so the gap is exact in floating point
            dd = trial[k] - trial[i]
            dist = math.hypot(dd[0], dd[1])
            target = radii[i] + radii[k] + g_min
            corr = 0.5 * (dist - target)
            uu = dd / dist
            trial[i] += corr * uu
            trial[k] -= corr * uu
            return trial
    raise RuntimeError("could not set the closest gap exactly")


def _mc_sweeps(c, radii, box, g_min, step, sweeps, rng):
    """Accept/reject Monte-Carlo sweeps (the packing randomisation of Sec. 6.2): each disk in
    turn proposes a displacement uniform in a disk of radius ``step``; it is accepted if the
    disk stays in the box and keeps gap >= g_min to every other disk."""
    P = c.shape[0]
    amax = radii.max()
    for _ in range(sweeps):
        tree = cKDTree(c)
        cand = tree.query_ball_point(c, r=2.0 * amax + g_min + 2.0 * step)
        rr = step * np.sqrt(rng.uniform(size=P))
        tt = rng.uniform(0.0, 2.0 * math.pi, size=P)
        disp = np.stack([rr * np.cos(tt), rr * np.sin(tt)], axis=1)
        for i in rng.permutation(P):
            p = c[i] + disp[i]
            if box is not None and (np.any(p < radii[i]) or np.any(p > box - radii[i])):
                continue
            nb = [k for k in cand[i] if k != i]
            if nb:
                nb = np.asarray(nb)
                d = np.hypot(c[nb, 0] - p[0], c[nb, 1] - p[1]) - radii[nb] - radii[i]
                if d.min() < g_min:
                    continue
            c[i] = p
    return c


def jittered_grid(seed, n=4, spacing=2.3, jitter=0.12, g_min=1e-3, radius=1.0):
    """n x n square grid with spacing ``spacing``, each centre jittered U[-jitter, jitter]^2.

    Pairs closer than g_min are pushed apart, then the closest pair is set to g_min.
    Returns (centres (P,2), radii (P,)).
    """
    rng = _rng(seed)
    ix, iy = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    c = np.stack([ix.ravel() * spacing, iy.ravel() * spacing], axis=1).astype(np.float64)
    c += rng.uniform(-jitter, jitter, size=c.shape)
    radii = np.full(c.shape[0], radius)
    c = _relax(c, radii, None, g_min * 1.02)
    c = _set_closest_gap(c, radii, g_min)
    return c, radii


def _triangular_sites(P, box, rng):
    nx = max(1, int(math.ceil(math.sqrt(P * math.sqrt(3.0) / 2.0))))
    ny = int(math.ceil(P / nx))
    sx = box / nx
    sy = box / ny
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    x = (ix + 0.5 + 0.25 * ((iy % 2) * 2 - 1)) * sx
    y = (iy + 0.5) * sy
    sites = np.stack([x.ravel(), y.ravel()], axis=1)
    if sites.shape[0] > P:
        keep = np.sort(rng.choice(sites.shape[0], size=P, replace=False))
        sites = sites[keep]
    lattice_gap_dist = min(sx, math.hypot(0.5 * sx, sy))
    return sites, lattice_gap_dist


def lattice_packing(seed, P, phi, g_min, rho, radius=1.0, sweeps=4):
    """Perturbed triangular lattice of P equal disks in a square box at area fraction phi.

    Each centre moves uniformly within a disk of radius rho*(s - 2a) (s the lattice
    distance), the packing is relaxed until every gap >= g_min, randomised by
    ``sweeps`` accept/reject Monte-Carlo sweeps (step (s - 2a)/2), and the closest
    pair is set to gap g_min exactly.  Returns (centres, radii, box side).
    """
    rng = _rng(seed)
    box = math.sqrt(P * math.pi * radius * radius / phi)
    sites, s = _triangular_sites(P, box, rng)
    amp = rho * max(s - 2.0 * radius, 0.0)
    r = amp * np.sqrt(rng.uniform(size=P))
    t = rng.uniform(0.0, 2.0 * math.pi, size=P)
    c = sites + np.stack([r * np.cos(t), r * np.sin(t)], axis=1)
    radii = np.full(P, radius)
    c = np.minimum(np.maximum(c, radius), box - radius)
    c = _relax(c, radii, box, g_min * 1.02)
    c = _mc_sweeps(c, radii, box, g_min * 1.02, 0.5 * max(s - 2.0 * radius, 0.05), sweeps, rng)
    c = _set_closest_gap(c, radii, g_min)
    return c, radii, box


def bidisperse_packing(seed, P, phi, g_min, rho, radii_pair=(1.0, 1.4)):
    """Triangular lattice with radii assigned 50/50 at random; perturb, relax, set closest gap."""
    rng = _rng(seed)
    radii = np.where(rng.uniform(size=P) < 0.5, radii_pair[0], radii_pair[1]).astype(np.float64)
    box = math.sqrt(math.pi * float(np.sum(radii * radii)) / phi)
    sites, s = _triangular_sites(P, box, rng)
    amp = rho * max(s - 2.0 * radii_pair[1], 0.0)
    r = amp * np.sqrt(rng.uniform(size=P))
    t = rng.uniform(0.0, 2.0 * math.pi, size=P)
    c = sites + np.stack([r * np.cos(t), r * np.sin(t)], axis=1)
    c = np.minimum(np.maximum(c, radii[:, None]), box - radii[:, None])
    c = _relax(c, radii, box, g_min * 1.02)
    c = _mc_sweeps(c, radii, box, g_min * 1.02, 0.5 * max(s - 2.0 * radii_pair[1], 0.05), 4, rng)
    c = _set_closest_gap(c, radii, g_min)
    return c, radii, box


# Perturbation amplitudes: C3's is calibrated so that the number of pairs with
# gap <= 0.2 is close to 0.99 P, the close-pair density of the paper's
# P = 10^4, area fraction 0.65 packing (9920 close pairs).
_RHO = {2: 0.9, 3: 1.62, 5: 0.9}


def config_geometry(cfg, k=0, P=None):
    """Geometry and discretisation parameters of the benchmark configurations.

    cfg 1: 16 disks, jittered 4x4 grid, min gap 1e-3, contact threshold 0.5.
    cfg 2: P = 1000, area fraction 0.5, min gap 1e-2.
    cfg 3: P = 10000, area fraction 0.65, min gap 1e-3.
    cfg 5: P = 20000 bidisperse (radii 1 and 1.4), area fraction 0.62, min gap 1e-4.
    ``P`` overrides the body count (same generator, same area fraction).
    Returns a dict of plain arrays and scalars.
    """
    seed = CONFIG_SEED_BASE + 1000 * cfg + k
    if cfg == 1:
        c, a = jittered_grid(seed)
        box = None
        delta_c = 0.5
        tol = 1e-8
    elif cfg == 2:
        c, a, box = lattice_packing(seed, P or 1000, 0.5, 1e-2, _RHO[2])
        delta_c = 0.2
        tol = 1e-6
    elif cfg == 3:
        c, a, box = lattice_packing(seed, P or 10000, 0.65, 1e-3, _RHO[3])
        delta_c = 0.2
        tol = 1e-7
    elif cfg == 5:
        c, a, box = bidisperse_packing(seed, P or 20000, 0.62, 1e-4, _RHO[5])
        delta_c = 0.2
        tol = 1e-7
    else:
        raise ValueError(f"unknown configuration {cfg}")
    n_src = np.where(a > 1.2, 50, 36).astype(np.int32)
    n_col = (2 * n_src).astype(np.int32)
    r_src = np.full(a.shape[0], 0.7)
    return dict(centers=np.ascontiguousarray(c, dtype=np.float64), radii=np.ascontiguousarray(a, dtype=np.float64),
                n_src=n_src, n_col=n_col, r_src=r_src, delta_c=delta_c, tol=tol, box=box, seed=seed)
