"""End-to-end parity on the GPU: device precompute + GMRES (FP64 and relaxed mixed) + post
against the FP64 oracle run independently (its own SVDs), on the 4x4 jittered grid
with min gap 1e-3 (contact threshold 0.5).

Tolerance 1e-9 on the relative residual (below the configuration's 1e-8; FP64
rounding of the resistance operator floors its true residual near 1e-10), except
resistance in mixed precision: its FP32 operator error (lubrication-sized
compressed strengths) slows the refinement, so it is run to 1e-6, the tolerance
of the resistance configuration.
Bar: max_i E^(i) <= 1e-5 (eq. rel_vel_err with the max-speed normalisation), the
accuracy the paper reports for its solves.  The per-pair matrices from two SVD
implementations agree to the truncation level, far below that.
"""

import numpy as np
import pytest

from oracle.pairs import pair_matrices
from oracle.params import MFSParams
from oracle.system import System, rel_rigid_error, solve
from workloads import jittered_grid, mobility_rhs, resistance_rhs
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

PRM = MFSParams(delta_c=0.5)


@pytest.fixture(scope="module")
def grid():
    c, a = jittered_grid(260611273 + 1000)
    return c, a


@pytest.mark.parametrize("problem", ["mobility", "resistance"])
def test_precompute_matches_oracle_pair_matrices(grid, problem):
    from paper_2606_11273_amd import native as nv
    c, a = grid
    prm = nv.mfs_default_params()
    prm.delta_c = 0.5
    ctx = nv.mfs_setup(c, a, 36, 72, 0.7, prm)
    try:
        say("precompute 4x4 grid", problem)
        n = nv.mfs_precompute_pairs(ctx, problem)
        As, Es = nv.mfs_get_pair_matrices(ctx, problem, np.full(16, 36))
        pr = nv.mfs_get_pairs(ctx)
        assert n == len(pr) >= 20
        S = System(c[:1], 1.0, 36, 72, 0.7, problem, PRM)  # one-body data only
        gaps = np.linalg.norm(c[pr[:, 1]] - c[pr[:, 0]], axis=1) - 2
        for p in np.unique(np.r_[np.argsort(gaps)[:3], np.argsort(gaps)[-2:]]):
            ref = pair_matrices(c[pr[p, 0]], c[pr[p, 1]], S.cls[0], PRM)
            ea = np.linalg.norm(As[p] - ref["A"]) / np.linalg.norm(ref["A"])
            ee = np.linalg.norm(Es[p] - ref["E"]) / np.linalg.norm(ref["E"])
            say(f"  pair {p} gap {gaps[p]:.2e}: |dA|/|A| = {ea:.2e}, |dE|/|E| = {ee:.2e}")
            assert ea < 1e-6 and ee < 1e-6
    finally:
        nv.mfs_destroy(ctx)


@pytest.mark.parametrize("problem", ["mobility", "resistance"])
def test_solve_matches_oracle(grid, problem):
    from paper_2606_11273_amd import native as nv
    c, a = grid
    given = mobility_rhs(260611273 + 1000, 16) if problem == "mobility" else resistance_rhs(260611273 + 1000, 16)
    S = System(c, a, 36, 72, 0.7, problem, PRM)
    ref, _, rinfo = solve(S, given, 1e-9)
    prm = nv.mfs_default_params()
    prm.delta_c = 0.5
    ctx = nv.mfs_setup(c, a, 36, 72, 0.7, prm)
    try:
        nv.mfs_precompute_pairs(ctx, problem)
        for prec in ("fp64", "mixed"):
            say("solve 4x4 grid", problem, prec)
            tol = 1e-6 if (problem, prec) == ("resistance", "mixed") else 1e-9
            out, info = nv.mfs_gmres_solve(ctx, problem, prec, given, tol, 300)
            E = rel_rigid_error(out, ref).max()
            say(f"  iters {info['iters']} (oracle {rinfo['iters']}), outer {info['outer']}, "
                f"resid {info['rel_resid']:.2e}, max E {E:.2e}")
            assert info["rel_resid"] <= tol
            assert E <= 1e-5
            if prec == "fp64":
                assert abs(info["iters"] - rinfo["iters"]) <= 2
    finally:
        nv.mfs_destroy(ctx)
