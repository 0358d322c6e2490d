"""Parity of the all-pairs Stokeslet sum (step 2a of Alg. 3, eq. getall) with the FP64 oracle.

Tolerances are stated per target relative to the magnitude
m_t = sum_s (|log r_ts| + 1) |sigma_s| / (4 pi mu), which bounds how rounding in the
terms can show in u_t: FP64 <= 1e-13 m_t; mixed (FP32 terms on body-relative
coordinates, FP64 accumulation over bodies) <= 2e-6 m_t, i.e. about 30 units in
the last place of FP32 per term.
"""

import numpy as np
import pytest
import torch

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
    assert np.all(np.abs(g["fp64"] - ref).max(1) <= 1e-13 * mag)
    assert np.all(np.abs(g["mixed"] - ref).max(1) <= 2e-6 * mag)


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
    assert np.all(np.abs(g["fp64"] - ref).max(1) <= 1e-13 * mag)
    assert np.all(np.abs(g["mixed"] - ref).max(1) <= 2e-6 * mag)


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
    assert np.all(np.abs(g["fp64"][tsel] - ref).max(1) <= 1e-13 * mag)
    assert np.all(np.abs(g["mixed"][tsel] - ref).max(1) <= 2e-6 * mag)


def test_kernel_sum_clusters_mid_size():
    # P = 600 packing at area fraction 0.5 (about 55 x 55): the FP32 sum takes the clusters
    # far from a target (beyond 4 cluster radii) from their expansions; 1500 sampled targets
    # against the oracle, and the clusters are a valid partition of the disks
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
        say(f"  skip {skip}: mixed max err / m_t {(np.abs(g['mixed'][tsel] - ref).max(1) / mag).max():.1e}")
        assert np.all(np.abs(g["fp64"][tsel] - ref).max(1) <= 1e-13 * mag)
        assert np.all(np.abs(g["mixed"][tsel] - ref).max(1) <= 2e-6 * mag)
