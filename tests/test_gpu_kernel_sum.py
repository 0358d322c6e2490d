"""Parity of the all-pairs Stokeslet sum (step 2a of Alg. 3, eq. getall) with the FP64 oracle.

Tolerances are stated per target relative to the magnitude
m_t = sum_s (|log r_ts| + 1) |sigma_s| / (4 pi mu), which bounds how rounding in the
terms can show in u_t: FP64 <= 1e-13 m_t everywhere; mixed (near disks' ring expansions in
FP32 from FP64 moments, FP64 accumulation; cell translations, local expansions and direct sums
in FP64) per case at about ten times the error measured on the MI355X (stated beside each
bound), so that a regression of an order of magnitude fails.
"""

import numpy as np
import pytest
import torch

import bench

from workloads import config_geometry, jittered_grid
from tests.gpu_helpers import coarse_points, oracle_sum_excluding_self, say

pytestmark = pytest.mark.gpu


def _run(centers, radii, n_src, n_col, r_src, sig, skip, delta_c=0.2):
    from paper_2606_11273_amd import native as nv
    prm = nv.mfs_default_params()
    prm.delta_c = delta_c
    ctx = nv.mfs_setup(centers, radii, n_src, n_col, r_src, prm)
    try:
        P, Ns, Nt, _ = nv.mfs_get_sizes(ctx)
        s = torch.tensor(sig.reshape(-1), dtype=torch.float64, device="cuda")
        out = {}
        for prec in ("fp64", "mixed"):
            u = torch.zeros(2 * Nt, dtype=torch.float64, device="cuda")
            nv.mfs_kernel_sum(ctx, prec, s, u, skip)
            torch.cuda.synchronize()
            out[prec] = u.cpu().numpy().reshape(-1, 2)
        return out
    finally:
        nv.mfs_destroy(ctx)


def _check(g, ref, mag, what, bound32, rows=slice(None)):
    e64 = (np.abs(g["fp64"][rows] - ref).max(1) / mag).max()
    e32 = (np.abs(g["mixed"][rows] - ref).max(1) / mag).max()
    say(f"  {what}: max err / m_t fp64 {e64:.2e} mixed {e32:.2e} (bound {bound32:.0e})")
    assert e64 <= 1e-13
    assert e32 <= bound32


def _partners(c, a, delta_c):
    from oracle.geometry import contacts
    nb = [set() for _ in range(len(c))]
    for i, k in contacts(c, a, delta_c):
        nb[i].add(int(k))
        nb[k].add(int(i))
    return nb


@pytest.mark.parametrize("skip", [0, 1, 2])
def test_kernel_sum_jittered_grid(skip):
    c, a = jittered_grid(260611273 + 1000)
    P = c.shape[0]
    ns, nc, rs = np.full(P, 36), np.full(P, 72), np.full(P, 0.7)
    X, Y, so, co = coarse_points(c, a, ns, nc, rs)
    sig = np.random.default_rng(0).standard_normal((Y.shape[0], 2))
    say("kernel sum 4x4 grid skip", skip)
    g = _run(c, a, ns, nc, rs, sig, skip, delta_c=0.5)
    ref, mag = oracle_sum_excluding_self(X, Y, sig, so, co, include_self=(skip == 0),
                                         partners=_partners(c, a, 0.5) if skip == 2 else None)
    _check(g, ref, mag, f"4x4 grid skip {skip}", 6e-8)   # measured 5.5e-9 .. 6.3e-9


def test_kernel_sum_ragged_mixed_classes():
    # 37 disks (ragged against every tile size), two disk classes with different counts
    rng = np.random.default_rng(1)
    c = np.stack(np.meshgrid(np.arange(7) * 3.1, np.arange(6) * 2.9), -1).reshape(-1, 2)[:37]
    c = c + rng.uniform(-0.2, 0.2, c.shape)
    a = np.where(np.arange(37) % 3 == 0, 1.0, 1.2)
    ns = np.where(a > 1.1, 50, 36)
    nc = 2 * ns
    rs = np.full(37, 0.7)
    X, Y, so, co = coarse_points(c, a, ns, nc, rs)
    sig = rng.standard_normal((Y.shape[0], 2))
    say("kernel sum ragged two classes")
    g = _run(c, a, ns, nc, rs, sig, 2, delta_c=1.0)
    ref, mag = oracle_sum_excluding_self(X, Y, sig, so, co, partners=_partners(c, a, 1.0))
    _check(g, ref, mag, "ragged two classes", 2e-8)   # measured 2.2e-9


def test_kernel_sum_full_size_sampled():
    # P = 10^4 packing at area fraction 0.65: 3.6e5 sources x 7.2e5 targets, the
    # launch configuration of the benchmark; the oracle evaluates 300 sampled targets.
    g0 = config_geometry(3)
    c, a = g0["centers"], g0["radii"]
    P = c.shape[0]
    ns, nc, rs = g0["n_src"], g0["n_col"], g0["r_src"]
    X, Y, so, co = coarse_points(c, a, ns, nc, rs)
    rng = np.random.default_rng(2)
    sig = rng.standard_normal((Y.shape[0], 2))
    say("kernel sum P=10000 sampled")
    g = _run(c, a, ns, nc, rs, sig, 2)
    tsel = np.sort(rng.choice(X.shape[0], 300, replace=False))
    tsel[0], tsel[-1] = 0, X.shape[0] - 1
    ref, mag = oracle_sum_excluding_self(X, Y, sig, so, co, targets=tsel, partners=_partners(c, a, 0.2))
    _check(g, ref, mag, "P=10000 sampled", 2e-9, tsel)   # measured 1.4e-10


def test_kernel_sum_clusters_mid_size():
    # P = 600 packing at area fraction 0.5 (about 55 x 55), where most of the (target, cell)
    # pairs are far: the hierarchical sum translates far cells into local expansions and takes
    # near disks from their ring expansions; 1500 sampled targets against the oracle.  The
    # clusters of the two-level sum at arbitrary points (mfs_get_clusters) are checked as a
    # partition of the disks
    from paper_2606_11273_amd import native as nv
    g0 = config_geometry(2, P=600)
    c, a = g0["centers"], g0["radii"]
    P = c.shape[0]
    ns, nc, rs = g0["n_src"], g0["n_col"], g0["r_src"]
    prm = nv.mfs_default_params()
    prm.delta_c = g0["delta_c"]
    ctx = nv.mfs_setup(c, a, ns, nc, rs, prm)
    try:
        cl = nv.mfs_get_clusters(ctx)
    finally:
        nv.mfs_destroy(ctx)
    order, st = cl["slot_body"], cl["cl_start"]
    assert np.array_equal(np.sort(order), np.arange(P)) and st[0] == 0 and st[-1] == P
    sizes = np.diff(st)
    assert sizes.min() >= 1 and sizes.max() <= 16
    for q in range(sizes.size):
        mem = order[st[q]:st[q + 1]]
        assert ns[mem].sum() <= 1024
        assert np.allclose(cl["centre"][q], c[mem].mean(0), rtol=0, atol=1e-12)
        assert np.all(np.linalg.norm(c[mem] - cl["centre"][q], axis=1) + rs[mem] * a[mem] <= cl["radius"][q] * (1 + 1e-15))
    X, Y, so, co = coarse_points(c, a, ns, nc, rs)
    d = np.linalg.norm(X[:, None, :] - cl["centre"][None, :, :], axis=2)
    far = d > 4 * cl["radius"][None, :]
    say(f"P=600: {sizes.size} clusters, mean radius {cl['radius'].mean():.2f}; "
        f"{far.mean():.2f} of the (target, cluster) pairs are far")
    assert far.mean() > 0.3
    rng = np.random.default_rng(3)
    sig = rng.standard_normal((Y.shape[0], 2))
    for skip in (0, 2):
        g = _run(c, a, ns, nc, rs, sig, skip, delta_c=g0["delta_c"])
        tsel = np.sort(rng.choice(X.shape[0], 1500, replace=False))
        ref, mag = oracle_sum_excluding_self(X, Y, sig, so, co, targets=tsel, include_self=(skip == 0),
                                             partners=_partners(c, a, g0["delta_c"]) if skip == 2 else None)
        _check(g, ref, mag, f"P=600 skip {skip}", 7e-9, tsel)   # measured 6.5e-10 .. 6.9e-10


def test_kernel_sum_projected_strengths():
    # the strengths the mobility matvec sums: N(0,1) per source, projected by (I - L) per disk
    # so that every disk carries zero net force and torque (Sec. 4.4).  Their fields cancel to
    # leading order at a distance; the mixed sum's ring expansions come from FP64 moments, so
    # its error stays relative to the field itself.  Dense-packing generator
    # (area fraction 0.65, min gap 1e-3) at P = 1000, 1500 sampled targets, skip mode 2.
    from oracle.onebody import one_body
    g0 = config_geometry(3, P=1000)
    c, a = g0["centers"], g0["radii"]
    ns, nc, rs = g0["n_src"], g0["n_col"], g0["r_src"]
    X, Y, so, co = coarse_points(c, a, ns, nc, rs)
    ob = one_body(1.0, 36, 72, 0.7, 1.0, "mobility", 1e-14, 1e-12)
    rng = np.random.default_rng(4)
    sig = np.concatenate([ob.project(rng.standard_normal(72)) for _ in range(c.shape[0])]).reshape(-1, 2)
    say("kernel sum projected strengths, dense packing P=1000")
    g = _run(c, a, ns, nc, rs, sig, 2)
    tsel = np.sort(rng.choice(X.shape[0], 1500, replace=False))
    ref, mag = oracle_sum_excluding_self(X, Y, sig, so, co, targets=tsel, partners=_partners(c, a, 0.2))
    field = np.abs(ref).max()
    e32 = np.abs(g["mixed"][tsel] - ref).max() / field
    say(f"  mixed: max err / max |u| {e32:.2e}; max |u| / max m_t {field / mag.max():.2e}")
    _check(g, ref, mag, "projected strengths", 3e-10, tsel)   # measured 2.2e-11
    assert e32 <= 3e-6   # measured 2.3e-7 of max |u|


def test_fmm_lists_partition_the_disks():
    # every wave's M2L cells and near disks cover each disk once; every M2L cell is separated
    # from the wave (|C - B| >= sep (R + r)) and holds no node's own disk or contact partner;
    # cells are quadtree ranges of the slot order with their centres and radii
    from paper_2606_11273_amd import native as nv
    g0 = config_geometry(2, P=600)
    c, a = g0["centers"], g0["radii"]
    ns, nc, rs = g0["n_src"], g0["n_col"], g0["r_src"]
    prm = nv.mfs_default_params()
    prm.delta_c = g0["delta_c"]
    X, Y, so, co = coarse_points(c, a, ns, nc, rs)
    ctx = nv.mfs_setup(c, a, ns, nc, rs, prm)
    try:
        cl = nv.mfs_get_clusters(ctx)
        pr = nv.mfs_get_pairs(ctx)
        f = {prec: nv.mfs_get_fmm(ctx, "mobility", prec) for prec in ("fp64", "mixed")}
    finally:
        nv.mfs_destroy(ctx)
    P = c.shape[0]
    sb = cl["slot_body"]
    slot_of = np.empty(P, dtype=int)
    slot_of[sb] = np.arange(P)
    partners = [set() for _ in range(P)]
    for i, k in pr:
        partners[i].add(int(k))
        partners[k].add(int(i))
    tp = bench.visiting_order(nc, sb)
    body_of_t = np.repeat(np.arange(P), nc)
    for prec, sep in (("fp64", 3.0), ("mixed", 2.0)):
        d = f[prec]
        lo, hi = d["cell_lo"], d["cell_hi"]
        assert np.array_equal(lo[:P], np.arange(P)) and np.array_equal(hi[:P], np.arange(1, P + 1))
        for q in range(len(lo)):
            mem = sb[lo[q]:hi[q]]
            C = c[mem].mean(0)
            assert np.allclose(d["cell_c"][q], C, atol=1e-12)
            assert d["cell_r"][q] >= (np.linalg.norm(c[mem] - C, axis=1) + a[mem]).max()
        ws = d["wave_start"]
        assert ws[0] == 0 and ws[-1] == X.shape[0] and np.all(np.diff(ws) >= 1) and np.all(np.diff(ws) <= 128)
        for w in range(len(ws) - 1):
            t = tp[ws[w]:ws[w + 1]]
            B = d["wave_c"][w]
            r = np.linalg.norm(X[t] - B, axis=1).max()
            excl = set()
            for b in set(body_of_t[t]):
                excl.add(slot_of[b])
                excl.update(slot_of[k] for k in partners[b])
            cover = np.zeros(P, dtype=int)
            for q in d["m2l"][d["m2l_off"][w]:d["m2l_off"][w + 1]]:
                assert np.linalg.norm(d["cell_c"][q] - B) >= sep * (d["cell_r"][q] + r) * (1 - 1e-12)
                assert not any(lo[q] <= e < hi[q] for e in excl)
                cover[lo[q]:hi[q]] += 1
            near = d["near"][d["near_off"][w]:d["near_off"][w + 1]]
            assert np.all(np.diff(near) > 0)
            cover[near] += 1
            assert np.all(cover == 1), (prec, w)


def _fmm_work(c, X, ns, nc, d, tp, partners, slot_of, mixed):
    """Host count of the kernel's rules per wave: the M2L list length (one translation, one
    wave), the local evaluations (64 lanes x 2 node slots per wave with translations) and, per
    near disk, the node slots of the 64 x 2 that take the lowest tier order whose squared
    distance every node not skipped (own disk and partners, skip mode 2) exceeds, else the
    direct sum over the disk's sources."""
    P = c.shape[0]
    sb = np.argsort(slot_of)
    body_of_t = np.repeat(np.arange(P), nc)
    orders = (14, 24, 44) if mixed else (27, 40, 56)
    thr = d["tier_d2"].copy()
    if mixed:   # the FP32 records hold the distances rounded up to FP32
        t32 = thr.astype(np.float32)
        t32 = np.where(t32.astype(np.float64) < thr, np.nextafter(t32, np.float32(np.inf)), t32)
        thr = t32.astype(np.float64)
    direct = exps = terms = m2l = l2p = 0
    ws = d["wave_start"]
    for w in range(len(ws) - 1):
        t = tp[ws[w]:ws[w + 1]]
        nm = d["m2l_off"][w + 1] - d["m2l_off"][w]
        m2l += nm
        l2p += 128 if nm > 0 else 0
        tb = body_of_t[t]
        for s in d["near"][d["near_off"][w]:d["near_off"][w + 1]]:
            b = sb[s]
            skip = np.array([b == bb or b in partners[bb] for bb in tb])
            if skip.all():
                continue
            r2 = ((X[t] - c[b]) ** 2).sum(1)
            p = 0
            for tier in range(3):
                if np.all(skip | (r2 > thr[s, tier])):
                    p = orders[tier]
                    break
            if p:
                exps += 128
                terms += 128 * p
            else:
                direct += 128 * ns[b]
    return direct, exps, terms, m2l, l2p


def test_kernel_sum_work_counters():
    # the kernels' own work counters (mfs_kernel_sum_work) against a host count of their rules
    # on the lists mfs_get_fmm exports, per launch, at P = 600 (area fraction 0.5), skip mode 2
    from paper_2606_11273_amd import native as nv
    g0 = config_geometry(2, P=600)
    c, a = g0["centers"], g0["radii"]
    ns, nc, rs = g0["n_src"], g0["n_col"], g0["r_src"]
    prm = nv.mfs_default_params()
    prm.delta_c = g0["delta_c"]
    X, Y, so, co = coarse_points(c, a, ns, nc, rs)
    ctx = nv.mfs_setup(c, a, ns, nc, rs, prm)
    try:
        cl = nv.mfs_get_clusters(ctx)
        pr = nv.mfs_get_pairs(ctx)
        fm = {prec: nv.mfs_get_fmm(ctx, "resistance", prec) for prec in ("fp64", "mixed")}
        s = torch.tensor(np.random.default_rng(5).standard_normal(2 * Y.shape[0]), device="cuda")
        u = torch.zeros(2 * X.shape[0], dtype=torch.float64, device="cuda")
        nv.mfs_kernel_sum_work(ctx, reset=True)
        counts = {}
        for prec in ("mixed", "fp64"):
            nv.mfs_kernel_sum(ctx, prec, s, u, 2)
            counts[prec] = nv.mfs_kernel_sum_work(ctx, reset=True)
    finally:
        nv.mfs_destroy(ctx)
    P = c.shape[0]
    slot_of = np.empty(P, dtype=int)
    slot_of[cl["slot_body"]] = np.arange(P)
    partners = [set() for _ in range(P)]
    for i, k in pr:
        partners[i].add(int(k))
        partners[k].add(int(i))
    tp = bench.visiting_order(nc, cl["slot_body"])
    say(f"work per launch: mixed {counts['mixed']}, fp64 {counts['fp64']}")
    for prec in ("mixed", "fp64"):
        ref = _fmm_work(c, X, ns, nc, fm[prec], tp, partners, slot_of, prec == "mixed")
        say(f"  host count {prec}: {ref}")
        assert ref[1] > 0 and ref[3] > 0
        assert tuple(counts[prec]) == ref, prec
