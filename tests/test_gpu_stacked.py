"""Stacked right-hand sides: the matvec on R vectors at once and the lockstep GMRES.

mfs_apply with n_rhs = R runs the stacked kernels (the geometry of each Stokeslet pair
evaluated once for all R strengths; each A^c read once for all R), in groups of 8, 4
and 2 with a single remainder through the one-vector path.  mfs_gmres_solve with
n_rhs = R runs R GMRES processes in lockstep on those stacked products.

Checks, on the 4x4 grid (min gap 1e-3) with the oracle's pair matrices imported:
* each stacked product equals the one-vector product: FP64 to 1e-12 of max |T mu| (the
  same terms; measured equal), mixed to the same bound as the one-vector mixed
  operator against the oracle (1e-5 mobility, 5e-3 resistance, smooth input), and the
  FP64 stacked product matches the oracle's Alg. 3 to 2e-11 for mobility and 1e-10 for
  resistance (whose compressed strengths are ~10^3 times the input near the gap-1e-3
  pairs and nearly cancel between the two disks, so FP64 rounding shows 3e2 times
  larger; 4e-11 measured);
* lockstep solves of 3 and 8 right-hand sides match solves of each one alone (both to
  the same relative residual tol: agreement 100 tol of max |v| + |omega|) and the
  oracle's solve (eq. rel_vel_err <= 1e-5).  tol is 1e-10 for mobility and 1e-6 for
  resistance: with these reduced fine grids (N_fp = 60) the oracle's own FP64 resistance
  solve stalls at a true residual of 5e-8 .. 9e-8 for these right-hand sides.
"""

import numpy as np
import pytest
import torch

from oracle.params import MFSParams
from oracle.system import System, rel_rigid_error, solve
from workloads import jittered_grid, mobility_rhs, resistance_rhs
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

SMALL = MFSParams(n_fp=60, n_ell=30, m_p=100, delta_c=0.5)


def _ctx(S, problem):
    from paper_2606_11273_amd import native as nv
    prm = nv.mfs_default_params()
    prm.delta_c = S.prm.delta_c
    ctx = nv.mfs_setup(S.c, S.a, S.n_src, S.n_col, S.r_src, prm)
    nv.mfs_set_pair_matrices(ctx, problem, [d["A"] for d in S.pd], [d["E"] for d in S.pd])
    return nv, ctx


def _given(problem, seed, P):
    return mobility_rhs(seed, P) if problem == "mobility" else resistance_rhs(seed, P)


@pytest.mark.parametrize("problem", ["mobility", "resistance"])
def test_stacked_matvec_equals_single(problem):
    c, a = jittered_grid(260611273 + 1000)
    S = System(c, a, 36, 72, 0.7, problem, SMALL)
    nv, ctx = _ctx(S, problem)
    try:
        for R in (8, 3):
            mus = np.stack([S.rhs(_given(problem, 40 + r, S.P)) for r in range(R)])
            refs = np.stack([S.matvec(m) for m in mus])
            dmu = torch.tensor(mus.reshape(-1), device="cuda")
            for prec in ("fp64", "mixed"):
                u = torch.zeros_like(dmu)
                nv.mfs_apply(ctx, problem, prec, dmu, u, n_rhs=R)
                torch.cuda.synchronize()
                stacked = u.cpu().numpy().reshape(R, -1)
                single = np.empty_like(stacked)
                for r in range(R):
                    ur = torch.zeros(S.n, dtype=torch.float64, device="cuda")
                    nv.mfs_apply(ctx, problem, prec, torch.tensor(mus[r], device="cuda"), ur)
                    torch.cuda.synchronize()
                    single[r] = ur.cpu().numpy()
                scale = np.abs(refs).max(axis=1)
                d_single = (np.abs(stacked - single).max(axis=1) / scale).max()
                d_oracle = (np.abs(stacked - refs).max(axis=1) / scale).max()
                say(f"stacked {problem} R={R} {prec}: vs one-vector {d_single:.2e}, vs oracle {d_oracle:.2e}")
                if prec == "fp64":
                    assert d_single <= 1e-12 and d_oracle <= (2e-11 if problem == "mobility" else 1e-10)
                else:
                    assert d_oracle <= (1e-5 if problem == "mobility" else 5e-3)
    finally:
        nv.mfs_destroy(ctx)


@pytest.mark.parametrize("problem", ["mobility", "resistance"])
def test_lockstep_solve_equals_single_solves(problem):
    c, a = jittered_grid(260611273 + 1000)
    S = System(c, a, 36, 72, 0.7, problem, SMALL)
    nv, ctx = _ctx(S, problem)
    try:
        for R in (3, 8):
            given = np.stack([_given(problem, 60 + r, S.P) for r in range(R)])
            for prec in ("fp64", "mixed"):
                tol = 1e-10 if problem == "mobility" else 1e-6
                out, info = nv.mfs_gmres_solve(ctx, problem, prec, given, tol, 300)
                alone = np.stack([nv.mfs_gmres_solve(ctx, problem, prec, given[r], tol, 300)[0] for r in range(R)])
                d = max(rel_rigid_error(out[r], alone[r]).max() for r in range(R))
                say(f"lockstep {problem} R={R} {prec}: iters {info['iters']} outer {info['outer']} "
                    f"resid {info['rel_resid']:.2e}; vs alone {d:.2e}")
                assert info["rel_resid"] <= tol
                assert d <= 100 * tol
        ref, _, _ = solve(S, given[0], 1e-9 if problem == "mobility" else 1e-7)
        E = rel_rigid_error(out[0], ref).max()
        say(f"  first right-hand side vs oracle: {E:.2e}")
        assert E <= 1e-5
    finally:
        nv.mfs_destroy(ctx)
