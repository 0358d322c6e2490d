"""The benchmark's work accounting (bench.ksum_work_clusters) against a brute-force count of
the kernel sums' rules.

The roofline's flops come from these counts.  A thread holds T = 2 targets, 256 apart in a
workgroup of 512; per cluster it takes the cluster's expansion when every target is beyond
4 cluster radii, else per disk of the cluster: the disk's expansion when every target is
beyond 7 ring radii, else the direct sum over its sources (both kernel sums).
16 x 16 disks on a jittered lattice of spacing 3 (18432 nodes, 36 workgroups), clusters of
2 x 2 disks, so that all three cases occur.
"""

import numpy as np

import bench


def _setup():
    rng = np.random.default_rng(7)
    g = np.stack(np.meshgrid(np.arange(16), np.arange(16), indexing="ij"), -1).reshape(-1, 2)
    c = g * 3.0 + rng.uniform(-0.2, 0.2, (256, 2))
    a = np.ones(256)
    ns, nc, rs = np.full(256, 36), np.full(256, 72), np.full(256, 0.7)
    # clusters: 2 x 2 blocks of the lattice
    blk = (g[:, 0] // 2) * 8 + g[:, 1] // 2
    order = np.argsort(blk, kind="stable").astype(np.int32)
    st = np.concatenate([[0], np.cumsum(np.bincount(blk))]).astype(np.int32)
    cen = np.array([c[order[st[q]:st[q + 1]]].mean(0) for q in range(64)])
    rad = np.array([(np.linalg.norm(c[order[st[q]:st[q + 1]]] - cen[q], axis=1) + 0.7).max() for q in range(64)])
    cl = dict(slot_body=order, cl_start=st, centre=cen, radius=rad)
    ang = 2 * np.pi * np.arange(72) / 72
    X = np.concatenate([c[i] + np.stack([np.cos(ang), np.sin(ang)], 1) for i in range(256)])
    return c, a, ns, rs, X, cl


def _brute(c, ns, rs, X, cl):
    P, T, B = c.shape[0], 2, 256
    nthr = X.shape[0] // (B * T) * B
    th = np.arange(nthr)
    tgt = np.stack([(th // B) * B * T + j * B + th % B for j in range(T)], 1)   # (threads, T)
    xt = X[tgt]                                                                   # (threads, T, 2)
    rho2 = (rs * 1.0) ** 2
    d2 = ((xt[:, :, None, :] - c[None, None, :, :]) ** 2).sum(-1)               # (threads, T, P)
    disk_far = (d2 > 49.0 * rho2[None, None, :]).all(1)                          # (threads, P)
    ncl = cl["radius"].size
    body_cl = np.empty(P, dtype=int)
    body_cl[cl["slot_body"]] = np.repeat(np.arange(ncl), np.diff(cl["cl_start"]))
    dc2 = ((xt[:, :, None, :] - cl["centre"][None, None, :, :]) ** 2).sum(-1)
    cl_far = (dc2 > 16.0 * cl["radius"][None, None, :] ** 2).all(1)              # (threads, ncl)
    near_b = ~cl_far[:, body_cl]                                                  # (threads, P)
    pairs32 = T * int(((near_b & ~disk_far) * ns[None, :]).sum())
    dexp32 = T * int((near_b & disk_far).sum())
    cexp32 = T * int(cl_far.sum())
    return pairs32, dexp32, cexp32


def test_work_counts_match_brute_force():
    c, a, ns, rs, X, cl = _setup()
    p32, d32, c32 = _brute(c, ns, rs, X, cl)
    assert min(d32, c32, p32) > 0
    assert bench.ksum_work_clusters(c, a, ns, rs, X, cl) == (p32, d32, c32)
