"""Edge cases of the GPU path: a single disk, no close pairs, a zero right-hand side, and
the largest disk discretisation the library accepts.

* One disk of radius a, viscosity mu (Sec. 3.1, the w = 0 frame of Remark 1): torque t
  turns it at omega = t / (4 pi mu a^2); force F moves it at F (1/2 - ln a) / (4 pi mu);
  resistance inverts these.  With one disk the all-pairs sum (own disk skipped) is empty,
  so both precisions give the FP64 answer: 1e-9 relative, as the oracle's own pin.
* Two disks farther apart than the contact threshold: no pairs, mfs_precompute_pairs
  returns 0, and the solve matches the oracle's (eq. rel_vel_err <= 1e-5).
* A zero right-hand side returns zeros after 0 iterations.
* n_src = 511, n_col = 512 (the largest ring sizes): the kernel sum in both precisions
  against the oracle's direct sum, to the bounds of the kernel-sum tests (1e-13 and 2e-6
  of sum_s (|log r| + 1) |sigma_s| / (4 pi mu)).
* An iteration limit below what the tolerance needs: MFS_ERR_NOCONV with the iterate's
  outputs written (finite, and within O(1) of the converged answer).
"""

import math

import numpy as np
import pytest
import torch

from oracle.params import MFSParams
from oracle.system import System, rel_rigid_error, solve
from tests.gpu_helpers import coarse_points, oracle_sum_excluding_self, say

pytestmark = pytest.mark.gpu


def _ctx(c, a, prm_mu=1.0, delta_c=0.2, ns=36, nc=72):
    from paper_2606_11273_amd import native as nv
    prm = nv.mfs_default_params()
    prm.mu = prm_mu
    prm.delta_c = delta_c
    return nv, nv.mfs_setup(c, a, ns, nc, 0.7, prm)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_single_disk_closed_forms(prec):
    for a, mu in ((1.0, 1.0), (1.4, 2.5)):
        nv, ctx = _ctx(np.array([[0.3, -0.7]]), a, mu)
        try:
            assert nv.mfs_precompute_pairs(ctx, "mobility") == 0
            assert nv.mfs_precompute_pairs(ctx, "resistance") == 0
            for ft in (np.array([0.0, 0.0, 1.0]), np.array([0.3, 0.9, -2.0])):
                out, info = nv.mfs_gmres_solve(ctx, "mobility", prec, ft[None], 1e-13, 100)
                v = ft[:2] * (0.5 - math.log(a)) / (4 * math.pi * mu)
                ref = np.array([v[0], v[1], ft[2] / (4 * math.pi * mu * a * a)])
                err = np.abs(out[0] - ref).max() / np.abs(ref).max()
                say(f"single disk a={a} mu={mu} {prec} mobility {ft}: err {err:.1e}, iters {info['iters']}")
                assert err <= 1e-9
            vw = np.array([0.2, -0.5, 0.8])
            out, _ = nv.mfs_gmres_solve(ctx, "resistance", prec, vw[None], 1e-13, 100)
            f = vw[:2] * 4 * math.pi * mu / (0.5 - math.log(a))
            ref = np.array([f[0], f[1], vw[2] * 4 * math.pi * mu * a * a])
            assert np.abs(out[0] - ref).max() <= 1e-9 * np.abs(ref).max()
        finally:
            nv.mfs_destroy(ctx)


def test_no_close_pairs_and_zero_rhs():
    c = np.array([[0.0, 0.0], [2.5, 0.4]])   # gap 0.53 > 0.2
    nv, ctx = _ctx(c, 1.0)
    try:
        assert nv.mfs_precompute_pairs(ctx, "mobility") == 0
        given = np.array([[0.4, -0.1, 1.0], [-0.4, 0.1, 0.3]])
        S = System(c, 1.0, 36, 72, 0.7, "mobility", MFSParams(delta_c=0.2))
        ref, _, _ = solve(S, given, 1e-12)
        for prec in ("fp64", "mixed"):
            out, info = nv.mfs_gmres_solve(ctx, "mobility", prec, given, 1e-12, 200)
            E = rel_rigid_error(out, ref).max()
            say(f"two far disks {prec}: iters {info['iters']}, max E {E:.1e}")
            assert E <= 1e-5
            zero, zinfo = nv.mfs_gmres_solve(ctx, "mobility", prec, np.zeros((2, 3)), 1e-12, 200)
            assert np.all(zero == 0.0) and zinfo["iters"] == 0 and zinfo["status"] == "MFS_OK"
    finally:
        nv.mfs_destroy(ctx)


def test_kernel_sum_largest_rings():
    from paper_2606_11273_amd import native as nv
    c = np.array([[0.0, 0.0], [2.6, 0.3], [1.1, 2.7]])
    a = np.ones(3)
    ns, nc, rs = np.full(3, 511), np.full(3, 512), np.full(3, 0.7)
    X, Y, so, co = coarse_points(c, a, ns, nc, rs)
    sig = np.random.default_rng(7).standard_normal((Y.shape[0], 2))
    prm = nv.mfs_default_params()
    prm.delta_c = 0.0
    ctx = nv.mfs_setup(c, a, ns, nc, rs, prm)
    try:
        for skip in (0, 1):
            ref, mag = oracle_sum_excluding_self(X, Y, sig, so, co, include_self=(skip == 0))
            for prec, tol in (("fp64", 1e-13), ("mixed", 2e-6)):
                u = torch.zeros(2 * X.shape[0], dtype=torch.float64, device="cuda")
                nv.mfs_kernel_sum(ctx, prec, torch.tensor(sig.reshape(-1), device="cuda"), u, skip)
                torch.cuda.synchronize()
                err = (np.abs(u.cpu().numpy().reshape(-1, 2) - ref).max(1) / mag).max()
                say(f"largest rings skip {skip} {prec}: max err / m_t {err:.1e}")
                assert err <= tol
    finally:
        nv.mfs_destroy(ctx)


def test_iteration_limit_returns_best_iterate():
    # MFS_ERR_NOCONV: GMRES stops at max_iter above the tolerance, outputs hold the iterate
    from workloads import jittered_grid, mobility_rhs
    c, a = jittered_grid(260611273 + 1000)
    nv, ctx = _ctx(c, a, delta_c=0.5)
    try:
        nv.mfs_precompute_pairs(ctx, "mobility")
        given = mobility_rhs(3, 16)
        full, _ = nv.mfs_gmres_solve(ctx, "mobility", "fp64", given, 1e-10, 300)
        for prec in ("fp64", "mixed"):
            out, info = nv.mfs_gmres_solve(ctx, "mobility", prec, given, 1e-10, 3, allow_noconv=True)
            say(f"iteration limit {prec}: status {info['status']}, iters {info['iters']}, resid {info['rel_resid']:.2e}")
            assert info["status"] == "MFS_ERR_NOCONV" and info["iters"] <= 3 and info["rel_resid"] > 1e-10
            assert np.all(np.isfinite(out)) and np.abs(out).max() > 0
            assert rel_rigid_error(out, full).max() < 1.0
            with pytest.raises(nv.MFSError) as e:
                nv.mfs_gmres_solve(ctx, "mobility", prec, given, 1e-10, 3)
            assert e.value.code == nv.MFS_ERR_NOCONV
    finally:
        nv.mfs_destroy(ctx)
