"""Parity of the GPU matvec T mu (Alg. 3), RHS and post-processing with the FP64 oracle.

The GPU imports the oracle's pair matrices A^c, E^c (mfs_set_pair_matrices), so
these tests isolate the matvec arithmetic from SVD differences; the one-body
factors are factorised independently on each side.  The reference is both the
oracle's step-by-step Alg. 3 and its closed masked form.

Tolerances are relative to max |T mu| and depend on the input:
* smooth mu (the system's own right-hand side): FP64 2e-11, mixed 1e-5 for
  mobility.  Resistance mixed: 5e-3.  Its compressed pair strengths lambda_tilde
  carry the lubrication forces of the near-contact pairs (much larger than the
  one-body strengths, nearly cancelling between the two disks), and the FP32
  terms round to eps_32 of each strength;
* rough mu (i.i.d. normal): the one-body pseudoinverse (eq. howG+) is backward
  stable only, so lambda_bar = S_L^+ mu is amplified by up to ~1e3-1e5 and two
  correct factorisations differ by cond(S_L) eps_64 ~ 1e7 * 1e-16 relative in it:
  FP64 1e-6.  The FP32 kernel sum rounds every term to ~eps_32 |sigma_s| |log r|
  while the exact far field of such strengths cancels: mixed 0.1.
"""

import math

import numpy as np
import pytest
import torch

from oracle.params import MFSParams
from oracle.system import System
from workloads import jittered_grid, mobility_rhs, resistance_rhs
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

SMALL = MFSParams(n_fp=60, n_ell=30, m_p=100, delta_c=0.5)


def _gpu_ctx(S, problem):
    from paper_2606_11273_amd import native as nv
    P = S.P
    prm = nv.mfs_default_params()
    prm.delta_c = S.prm.delta_c
    ctx = nv.mfs_setup(S.c, S.a, S.n_src, S.n_col, S.r_src, prm)
    pr = nv.mfs_get_pairs(ctx)
    assert np.array_equal(pr, S.pairs.astype(np.int32).reshape(-1, 2)), "contact lists differ"
    nv.mfs_set_pair_matrices(ctx, problem, [d["A"] for d in S.pd], [d["E"] for d in S.pd])
    return nv, ctx


@pytest.mark.parametrize("problem", ["mobility", "resistance"])
def test_matvec_rhs_post_with_oracle_matrices(problem):
    c, a = jittered_grid(260611273 + 1000)
    S = System(c, a, 36, 72, 0.7, problem, SMALL)
    say("matvec 4x4 grid", problem, "pairs", len(S.pairs))
    nv, ctx = _gpu_ctx(S, problem)
    try:
        rng = np.random.default_rng(3)
        for trial in range(2):
            mu = S.rhs(mobility_rhs(5, S.P) if problem == "mobility" else resistance_rhs(5, S.P)) if trial == 0 \
                else rng.standard_normal(S.n)
            ref = S.matvec(mu)
            dmu = torch.tensor(mu, device="cuda")
            out = {}
            for prec in ("fp64", "mixed"):
                u = torch.zeros_like(dmu)
                nv.mfs_apply(ctx, problem, prec, dmu, u)
                torch.cuda.synchronize()
                out[prec] = u.cpu().numpy()
            refm = S.matvec_masked(mu)
            scale = np.abs(ref).max()
            e64 = np.abs(out["fp64"] - ref).max() / scale
            e64m = np.abs(out["fp64"] - refm).max() / scale
            e32 = np.abs(out["mixed"] - ref).max() / scale
            say(f"  trial {trial}: fp64 vs Alg.3 {e64:.2e}, vs masked {e64m:.2e}; mixed {e32:.2e}; "
                f"oracle Alg.3 vs masked {np.abs(ref - refm).max() / scale:.2e}")
            tol64, tol32 = (2e-11, 1e-5 if problem == "mobility" else 5e-3) if trial == 0 else (1e-6, 1e-1)
            assert e64 <= tol64 and e64m <= tol64
            assert e32 <= tol32
        # RHS and post-processing
        given = mobility_rhs(6, S.P) if problem == "mobility" else resistance_rhs(6, S.P)
        b = torch.zeros(S.n, dtype=torch.float64, device="cuda")
        nv.mfs_rhs(ctx, problem, given, b)
        bref = S.rhs(given)
        assert np.abs(b.cpu().numpy() - bref).max() <= 1e-12 * np.abs(bref).max()
        for mu, tol in ((bref, 1e-11), (rng.standard_normal(S.n), 1e-6)):
            post = nv.mfs_post(ctx, problem, torch.tensor(mu, device="cuda"), S.P)
            pref = S.post(mu)
            say(f"  post: {np.abs(post - pref).max() / np.abs(pref).max():.2e}")
            assert np.abs(post - pref).max() <= tol * np.abs(pref).max()
    finally:
        nv.mfs_destroy(ctx)


@pytest.mark.parametrize("problem", ["mobility", "resistance"])
def test_isolated_pair_is_identity_on_gpu(problem):
    from paper_2606_11273_amd import native as nv
    c = np.array([[0.3, -0.1], [0.3 + 2.001 * math.cos(0.9), -0.1 + 2.001 * math.sin(0.9)]])
    prm = nv.mfs_default_params()
    ctx = nv.mfs_setup(c, 1.0, 36, 72, 0.7, prm)
    try:
        say("isolated pair identity", problem)
        assert nv.mfs_precompute_pairs(ctx, problem) == 1
        b = torch.zeros(288, dtype=torch.float64, device="cuda")
        nv.mfs_rhs(ctx, problem, np.array([[0.3, -0.2, 1.0], [-0.3, 0.2, 0.4]]), b)
        rough = torch.tensor(np.random.default_rng(4).standard_normal(288), device="cuda")
        for mu, prec, tol in ((b, "fp64", 1e-12), (b, "mixed", 1e-6), (rough, "fp64", 1e-10), (rough, "mixed", 1e-1)):
            u = torch.zeros_like(mu)
            nv.mfs_apply(ctx, problem, prec, mu, u)
            torch.cuda.synchronize()
            err = (u - mu).abs().max().item() / mu.abs().max().item()
            say("  ", prec, "smooth" if mu is b else "rough", "max |T mu - mu| / max |mu| =", err)
            assert err <= tol
    finally:
        nv.mfs_destroy(ctx)


def test_apply_before_precompute_is_a_state_error():
    from paper_2606_11273_amd import native as nv
    c = np.array([[0.0, 0.0], [2.01, 0.0]])
    ctx = nv.mfs_setup(c, 1.0, 36, 72, 0.7)
    try:
        mu = torch.zeros(288, dtype=torch.float64, device="cuda")
        with pytest.raises(nv.MFSError) as e:
            nv.mfs_apply(ctx, "mobility", "fp64", mu, torch.zeros_like(mu))
        assert e.value.code == nv.MFS_ERR_STATE
    finally:
        nv.mfs_destroy(ctx)
