"""mfs_apply_noalloc (the matvec with no device allocation) against mfs_apply.

The no-allocation entry point keeps the kernel sum's expansion records (the disks' ring
expansions and the cells' moments) in the library's static scratch array instead of the
context's own buffers; everything else is the same launch sequence, so its output must equal
mfs_apply's bit for bit.  Two calls in a row on the same
device, the second on a smaller context (the array keeps the first call's contents), in both
precisions and both problems.  The pair matrices are seeded random ones of the right shapes
(the comparison is between two entry points on one operator).
A context whose records exceed the array is refused with MFS_ERR_ARG.
"""

import numpy as np
import pytest
import torch

from workloads import config_geometry, jittered_grid
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def _ctx(nv, c, a, ns, nc, rs, delta_c, seed):
    prm = nv.mfs_default_params()
    prm.delta_c = delta_c
    ctx = nv.mfs_setup(c, a, ns, nc, rs, prm)
    rng = np.random.default_rng(seed)
    pr = nv.mfs_get_pairs(ctx)
    sizes = [2 * int(ns[i] + ns[k]) for i, k in pr]
    for problem in ("mobility", "resistance"):
        nv.mfs_set_pair_matrices(ctx, problem, [1e-2 * rng.standard_normal((m, m)) for m in sizes],
                                 [rng.standard_normal((6, m)) for m in sizes])
    return ctx


def test_noalloc_equals_apply_two_calls():
    from paper_2606_11273_amd import native as nv
    g = config_geometry(3, P=2000)
    big = (g["centers"], g["radii"], g["n_src"], g["n_col"], g["r_src"], g["delta_c"])
    c, a = jittered_grid(260611273 + 1000)
    small = (c, a, np.full(16, 36), np.full(16, 72), np.full(16, 0.7), 0.5)
    for name, geo in (("P=2000 dense packing", big), ("4x4 grid", small)):
        ctx = _ctx(nv, *geo, seed=1)
        try:
            _, _, Nt, _ = nv.mfs_get_sizes(ctx)
            mu = torch.tensor(np.random.default_rng(2).standard_normal(2 * Nt), device="cuda")
            for problem in ("mobility", "resistance"):
                for prec in ("fp64", "mixed"):
                    u0 = torch.full_like(mu, np.nan)
                    u1 = torch.full_like(mu, np.nan)
                    nv.mfs_apply(ctx, problem, prec, mu, u0)
                    nv.mfs_apply_noalloc(ctx, problem, prec, mu, u1)
                    torch.cuda.synchronize()
                    d = (u1 - u0).abs().max().item()
                    say(f"{name} {problem} {prec}: max |noalloc - apply| = {d:.1e}")
                    assert torch.isfinite(u1).all()
                    assert torch.equal(u0, u1)
        finally:
            nv.mfs_destroy(ctx)


def test_noalloc_refuses_records_beyond_scratch():
    # 142 x 142 disks on a square lattice of spacing 3 (no close pairs, so no precompute): the
    # kernel sum's records need 16 (ncell (81 + 108) + 174 P) + 1120 P bytes, about 170 MB,
    # above the 128 MiB array
    from paper_2606_11273_amd import native as nv
    n = 142
    g = np.stack(np.meshgrid(np.arange(n), np.arange(n), indexing="ij"), -1).reshape(-1, 2) * 3.0
    P = g.shape[0]
    prm = nv.mfs_default_params()
    ctx = nv.mfs_setup(g.astype(np.float64), np.ones(P), np.full(P, 36), np.full(P, 72), np.full(P, 0.7), prm)
    try:
        assert nv.mfs_get_pairs(ctx).shape[0] == 0
        _, _, Nt, _ = nv.mfs_get_sizes(ctx)
        mu = torch.ones(2 * Nt, dtype=torch.float64, device="cuda")
        u = torch.zeros_like(mu)
        with pytest.raises(nv.MFSError) as e:
            nv.mfs_apply_noalloc(ctx, "mobility", "mixed", mu, u)
        assert e.value.code == nv.MFS_ERR_ARG
        say(f"refused: {e.value}")
    finally:
        nv.mfs_destroy(ctx)
