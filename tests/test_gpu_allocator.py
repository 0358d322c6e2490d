"""Contexts whose device memory comes from the caller's allocator (mfs_setup_ex).

Two contexts of the 4x4 jittered grid (min gap 1e-3, contact threshold 0.5), one with
hipMalloc and one with PyTorch's caching allocator through the callbacks, run the same
calls: pair precompute with fine factors, a 3-vector stacked product, a mixed solve of
two right-hand sides in lockstep, the density and the boundary residual.  The results
are bitwise equal (the arithmetic does not depend on where buffers live; every
reduction has a fixed order).  Through the callbacks: every allocation is freed by
mfs_destroy, and while the context lives its buffers are counted by PyTorch.
"""

import numpy as np
import pytest
import torch

from workloads import jittered_grid, mobility_rhs, unit_torques
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def _run(nv, ctx, P):
    nv.mfs_keep_fine_factors(ctx, True)
    nv.mfs_precompute_pairs(ctx, "mobility")
    _, _, Nt, _ = nv.mfs_get_sizes(ctx)
    n = 2 * Nt
    gen = torch.Generator(device="cpu").manual_seed(5)
    mu = torch.randn(3 * n, generator=gen, dtype=torch.float64).cuda()
    u = torch.zeros_like(mu)
    nv.mfs_apply(ctx, "mobility", "mixed", mu, u, n_rhs=3)
    given = np.stack([unit_torques(P), mobility_rhs(3, P)])
    out, info = nv.mfs_gmres_solve(ctx, "mobility", "mixed", given, 1e-10, 300)
    dens = torch.zeros(n, dtype=torch.float64, device="cuda")
    nv.mfs_get_density(ctx, 1, dens)
    em = nv.mfs_boundary_residual(ctx, "mobility", dens, given[1], out[1], 64)
    torch.cuda.synchronize()
    return dict(u=u.cpu().numpy(), out=out, dens=dens.cpu().numpy(), em=em, iters=info["iters"])


def test_torch_allocator_context_matches_and_releases():
    from paper_2606_11273_amd import native as nv
    c, a = jittered_grid(260611273 + 1000)
    prm = nv.mfs_default_params()
    prm.delta_c = 0.5
    ref_ctx = nv.mfs_setup(c, a, 36, 72, 0.7, prm)
    try:
        ref = _run(nv, ref_ctx, len(c))
    finally:
        nv.mfs_destroy(ref_ctx)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    alloc = nv.TorchAllocator()
    ctx = nv.mfs_setup(c, a, 36, 72, 0.7, prm, allocator=alloc)
    try:
        got = _run(nv, ctx, len(c))
        live = alloc.live_bytes
        say(f"torch allocator: {alloc.allocs} allocations, {alloc.frees} frees so far, {live / 2**20:.1f} MiB live; "
            f"torch counts {(torch.cuda.memory_allocated() - base) / 2**20:.1f} MiB above the baseline")
        assert alloc.allocs > 0 and live > 0
        assert torch.cuda.memory_allocated() - base >= live
    finally:
        nv.mfs_destroy(ctx)
    torch.cuda.synchronize()
    say(f"after destroy: {alloc.allocs} allocations, {alloc.frees} frees, {len(alloc.live)} live")
    assert alloc.frees == alloc.allocs and not alloc.live
    assert torch.cuda.memory_allocated() == base
    for key in ("u", "out", "dens"):
        assert np.array_equal(got[key], ref[key]), key
    assert got["em"] == ref["em"] and got["iters"] == ref["iters"]


def test_allocator_without_callbacks_is_an_argument_error():
    from paper_2606_11273_amd import native as nv

    class Broken:
        struct = nv.MfsAllocator()   # NULL callbacks

    c, a = jittered_grid(260611273 + 1000)
    with pytest.raises(nv.MFSError) as e:
        nv.mfs_setup(c, a, 36, 72, 0.7, allocator=Broken())
    assert e.value.code == nv.MFS_ERR_ARG
