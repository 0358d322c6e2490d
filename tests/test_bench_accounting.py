"""The benchmark's work accounting (bench.ksum_work_clusters) against a brute-force count of
the kernel sums' rules.

The kernels count their own work on the device (mfs_kernel_sum_work); these host counts pin
their rules.  A thread holds T = 2 consecutive targets of a workgroup's 512, and a wave of 64
threads takes one path for all of its 128 targets: per cluster the cluster's expansion when
every target is beyond 4 cluster radii, else per disk of the cluster the disk's expansion
when every target is beyond 7 ring radii, else the direct sum over its sources (both kernel
sums); with the local expansions, a cluster far from a whole workgroup's targets goes into the
workgroup's local expansion instead.  16 x 16 disks on a jittered lattice of spacing 3 (18432
nodes, 36 workgroups), clusters of 2 x 2 disks, so that every case occurs.
"""

import math

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


def _brute(c, ns, rs, X, cl, tperm=None, local=False, splits=1, sep=3.0):
    """Per wave (64 threads of T = 2 targets; thread tid of block b holds the targets at
    positions b 512 + 2 tid + j of the visiting order), the kernels' decisions taken for all
    its targets at once; with `local`, first per block: the clusters that go into the block's
    local expansion (beyond 4 R + rb and sep (R + rb) of the centre of its targets' bounding box,
    rb its half diagonal)."""
    P, T, B, W = c.shape[0], 2, 256, 64
    Nt = X.shape[0]
    nblk = -(-Nt // (B * T))
    pos = np.arange(nblk * B * T)
    tgt = np.minimum(pos, Nt - 1)
    if tperm is not None:
        tgt = tperm[tgt]
    b, r = pos // (B * T), pos % (B * T)
    tid, j = r // T, r % T
    assert np.array_equal(b * B * T + tid * T + j, pos)
    wave = b * (B // W) + tid // W
    order = np.argsort(wave, kind="stable")
    wt = tgt[order].reshape(-1, W * T)                                            # (waves, 128)
    xt = X[wt]
    ncl = cl["radius"].size
    # per block: bounding box of its 512 targets, then the local-expansion test per cluster
    le = np.zeros((nblk, ncl), dtype=bool)
    if local:
        for blk in range(nblk):
            pts = X[tgt[blk * B * T:(blk + 1) * B * T]]
            lo, hi = pts.min(0), pts.max(0)
            cen = (lo + hi) / 2
            rb = 0.5 * math.hypot(*(hi - lo)) * (1 + 1e-9) + 1e-9
            for q in range(ncl):
                R = cl["radius"][q]
                thr = max(4 * (1 + 1e-6) * R + rb, sep * (R + rb))
                le[blk, q] = math.hypot(*(cl["centre"][q] - cen)) > thr
    le_w = np.repeat(le, B // W, axis=0)                                          # (waves, ncl)
    rho2 = (rs * 1.0) ** 2
    d2 = ((xt[:, :, None, :] - c[None, None, :, :]) ** 2).sum(-1)               # (waves, 128, P)
    disk_far = (d2 > 49.0 * rho2[None, None, :]).all(1)                          # (waves, P)
    body_cl = np.empty(P, dtype=int)
    body_cl[cl["slot_body"]] = np.repeat(np.arange(ncl), np.diff(cl["cl_start"]))
    dc2 = ((xt[:, :, None, :] - cl["centre"][None, None, :, :]) ** 2).sum(-1)
    cl_far = (dc2 > 16.0 * cl["radius"][None, None, :] ** 2).all(1) & ~le_w     # (waves, ncl)
    near_b = ~(cl_far | le_w)[:, body_cl]                                         # (waves, P)
    lanes = W * T
    pairs32 = lanes * int(((near_b & ~disk_far) * ns[None, :]).sum())
    dexp32 = lanes * int((near_b & disk_far).sum())
    cexp32 = lanes * int(cl_far.sum())
    cps = -(-ncl // splits)
    evals = sum(B * T for blk in range(nblk) for s0 in range(0, ncl, cps) if le[blk, s0:s0 + cps].any())
    return pairs32, dexp32, cexp32, int(le.sum()), evals


def test_work_counts_match_brute_force():
    c, a, ns, rs, X, cl = _setup()
    ref = _brute(c, ns, rs, X, cl)
    assert min(ref[:3]) > 0 and ref[3:] == (0, 0)
    assert bench.ksum_work_clusters(c, a, ns, rs, X, cl, local=False) == ref


def test_work_counts_in_visiting_order_with_ragged_tail_and_local_expansions():
    # the targets visited disk by disk in the clusters' slot order, a node count that leaves a
    # partly filled last workgroup (clamped positions), and the workgroups' local expansions
    c, a, ns, rs, X, cl = _setup()
    X = X[:-100]
    nc = np.full(256, 72)
    tperm = bench.visiting_order(nc, cl["slot_body"])
    tperm = tperm[tperm < X.shape[0]]
    for splits, sep in ((1, 3.0), (4, 3.0), (4, 4.0)):
        ref = _brute(c, ns, rs, X, cl, tperm, local=True, splits=splits, sep=sep)
        assert min(ref) > 0
        assert bench.ksum_work_clusters(c, a, ns, rs, X, cl, tperm=tperm, local=True, splits=splits, sep=sep) == ref
    assert ref[:3] != _brute(c, ns, rs, X, cl, tperm)[:3]
