"""The no-allocation matvec recorded into a HIP graph and replayed.

Callers that cannot allocate, such as code under HIP graph capture, use mfs_apply_noalloc.  On a
context whose stream is the capturing stream its launches (no allocation, no copy, no fill, no
synchronisation) record into a graph.  Each replay, with new input copied into the captured
buffer and the program's own eager work and synchronisations in between, must equal the eager
mfs_apply of the same input bit for bit: the same kernels run in the same order.  Both problems
and both precisions, on the 16-disk grid with seeded random pair matrices of the right shapes
(the comparison is between two launch routes of one operator).
"""

import numpy as np
import pytest
import torch

from workloads import jittered_grid
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def test_noalloc_matvec_graph_replays():
    from paper_2606_11273_amd import native as nv
    c, a = jittered_grid(260611273 + 2000)
    ns, nc, rs = np.full(16, 36), np.full(16, 72), np.full(16, 0.7)
    s = torch.cuda.Stream()
    prm = nv.mfs_default_params()
    prm.delta_c = 0.5
    ctx = nv.mfs_setup(c, a, ns, nc, rs, prm, stream=s.cuda_stream)
    try:
        rng = np.random.default_rng(7)
        pr = nv.mfs_get_pairs(ctx)
        assert len(pr) > 0
        sizes = [2 * int(ns[i] + ns[k]) for i, k in pr]
        for problem in ("mobility", "resistance"):
            nv.mfs_set_pair_matrices(ctx, problem, [1e-2 * rng.standard_normal((m, m)) for m in sizes],
                                     [rng.standard_normal((6, m)) for m in sizes])
        _, _, Nt, _ = nv.mfs_get_sizes(ctx)
        for problem in ("mobility", "resistance"):
            for prec in ("fp64", "mixed"):
                mu_s = torch.zeros(2 * Nt, dtype=torch.float64, device="cuda")
                u_s = torch.zeros_like(mu_s)
                torch.cuda.synchronize()
                with torch.cuda.stream(s):   # first launches outside the capture (code objects load)
                    nv.mfs_apply_noalloc(ctx, problem, prec, mu_s, u_s)
                torch.cuda.synchronize()
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=s):
                    nv.mfs_apply_noalloc(ctx, problem, prec, mu_s, u_s)
                torch.cuda.synchronize()
                for rep in range(3):
                    x = torch.tensor(rng.standard_normal(2 * Nt), device="cuda")
                    mu_s.copy_(x)
                    u_s.fill_(float("nan"))
                    g.replay()
                    torch.cuda.synchronize()
                    got = u_s.clone()
                    ref = torch.full_like(x, float("nan"))
                    with torch.cuda.stream(s):
                        nv.mfs_apply(ctx, problem, prec, x, ref)
                    torch.cuda.synchronize()
                    d = (got - ref).abs().max().item()
                    say(f"{problem} {prec} replay {rep}: max |graph - eager| = {d:.1e}")
                    assert torch.isfinite(got).all()
                    assert torch.equal(got, ref)
                del g
                torch.cuda.synchronize()
    finally:
        nv.mfs_destroy(ctx)
