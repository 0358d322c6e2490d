"""Flow evaluation and boundary residual on the GPU against the oracle (oracle/flow.py).

Workload: the 4x4 jittered grid (min gap 1e-3, contact threshold 0.5, 23 close pairs),
N_c = 36 on radius 0.7, M_c = 72, the paper's fine parameters.  The oracle solves the
problem (FP64, tolerance 1e-12); both sides then evaluate the flow from that same density
mu (the GPU reads it from a device copy), with their own pair precompute:

* velocities at 64 boundary points per disk (with their disk), at fluid points across the
  gaps of the three closest pairs (inside their peanuts) and at 200 random fluid points:
  GPU against oracle elementwise to 1e-7 of max |u|.  The two sides factor the
  ill-conditioned fine and peanut matrices with different SVDs (truncations 1e-11 and
  1e-14), which leaves differences far below the method's own error (1e-3 .. 1e-5 here);
* the relative boundary residual eps_max on the same density: to 1e-7 (it is a ratio);
* end to end on the GPU: mixed solve, mfs_get_density, boundary residual of the GPU's own
  solution: within 1e-6 of the oracle's eps_max;
* state errors: flow evaluation without kept fine factors, density before any solve.
"""

import numpy as np
import pytest
import torch

from oracle.flow import boundary_residual, flow_eval
from oracle.geometry import contacts, perp
from oracle.pairs import pair_matrices
from oracle.params import MFSParams
from oracle.system import System, solve
from workloads import jittered_grid, mobility_rhs, resistance_rhs
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

PRM = MFSParams(delta_c=0.5)


def _oracle(problem, c, a):
    S0 = System(c, a, 36, 72, 0.7, problem, PRM, pair_data=[None] * len(contacts(c, a, PRM.delta_c)))
    full = [pair_matrices(S0.c[i], S0.c[k], S0.cls[i], PRM, keep=True, ob_k=S0.cls[k]) for i, k in S0.pairs]
    S = System(c, a, 36, 72, 0.7, problem, PRM, pair_data=[dict(A=d["A"], E=d["E"]) for d in full])
    fine = [dict(Yfi=d["Yfi"], Yfk=d["Yfk"], G=d["G"]) for d in full]
    return S, fine


def _points(S, rng):
    gaps = np.linalg.norm(S.c[S.pairs[:, 1]] - S.c[S.pairs[:, 0]], axis=1) - S.a[S.pairs[:, 0]] - S.a[S.pairs[:, 1]]
    pts = []
    for p in np.argsort(gaps)[:3]:
        i, k = S.pairs[p]
        e = (S.c[k] - S.c[i]) / np.linalg.norm(S.c[k] - S.c[i])
        mid = S.c[i] + (S.a[i] + 0.5 * gaps[p]) * e
        for h in (0.0, 0.003, -0.02, 0.1):
            pts.append(mid + h * perp(e))
    lo, hi = S.c.min(0) - 1.5, S.c.max(0) + 1.5
    while len(pts) < 12 + 200:
        x = lo + (hi - lo) * rng.uniform(size=2)
        if np.all(np.linalg.norm(S.c - x, axis=1) > S.a * 1.001):
            pts.append(x)
    fluid = np.array(pts)
    nb = 64
    th = (np.arange(nb) + 0.5) * (2 * np.pi / nb)
    ring = np.stack([np.cos(th), np.sin(th)], axis=1)
    bnd = np.concatenate([S.c[i] + S.a[i] * ring for i in range(S.P)])
    body = np.concatenate([np.repeat(np.arange(S.P), nb), -np.ones(len(fluid), dtype=np.int64)])
    return np.concatenate([bnd, fluid]), body


@pytest.mark.parametrize("problem", ["mobility", "resistance"])
def test_flow_and_residual_match_oracle(problem):
    from paper_2606_11273_amd import native as nv
    c, a = jittered_grid(260611273 + 1000)
    S, fine = _oracle(problem, c, a)
    given = mobility_rhs(7, 16) if problem == "mobility" else resistance_rhs(7, 16)
    out_or, mu_or, _ = solve(S, given, 1e-12)
    rigid = out_or if problem == "mobility" else given
    pts, body = _points(S, np.random.default_rng(2))
    ref = flow_eval(S, mu_or, pts, body, given=given, fine=fine)
    _, em_ref = boundary_residual(S, mu_or, rigid, 64, given=given, fine=fine)

    prm = nv.mfs_default_params()
    prm.delta_c = PRM.delta_c
    ctx = nv.mfs_setup(c, a, 36, 72, 0.7, prm)
    try:
        dmu = torch.tensor(mu_or, device="cuda")
        dpts = torch.tensor(pts.reshape(-1), device="cuda")
        dbody = torch.tensor(body, dtype=torch.int32, device="cuda")
        u = torch.zeros(2 * len(body), dtype=torch.float64, device="cuda")
        # state errors first: no solve yet, no fine factors yet
        with pytest.raises(nv.MFSError) as e:
            nv.mfs_get_density(ctx, 0, torch.zeros_like(dmu))
        assert e.value.code == nv.MFS_ERR_STATE
        nv.mfs_precompute_pairs(ctx, problem)
        with pytest.raises(nv.MFSError) as e:
            nv.mfs_flow_eval(ctx, problem, dmu, given, dpts, dbody, u)
        assert e.value.code == nv.MFS_ERR_STATE
        nv.mfs_keep_fine_factors(ctx, True)
        say(f"flow {problem}: precompute with fine factors, {len(S.pairs)} pairs")
        nv.mfs_precompute_pairs(ctx, problem)
        nv.mfs_flow_eval(ctx, problem, dmu, given, dpts, dbody, u)
        torch.cuda.synchronize()
        ug = u.cpu().numpy().reshape(-1, 2)
        scale = np.abs(ref).max()
        err = np.abs(ug - ref).max(axis=1) / scale
        nbnd = int(np.sum(body >= 0))
        say(f"  boundary points: max err {err[:nbnd].max():.2e}; gap points {err[nbnd:nbnd + 12].max():.2e}; "
            f"random fluid points {err[nbnd + 12:].max():.2e} (of max |u| {scale:.2e})")
        assert err.max() <= 1e-7
        eps = torch.zeros(16 * 64, dtype=torch.float64, device="cuda")
        em = nv.mfs_boundary_residual(ctx, problem, dmu, given, rigid, 64, eps)
        say(f"  eps_max GPU {em:.6e}, oracle {em_ref:.6e}")
        assert abs(em - em_ref) <= 1e-7
        # end to end: the GPU's own mixed solve and its density
        out, info = nv.mfs_gmres_solve(ctx, problem, "mixed", given, 1e-9 if problem == "mobility" else 1e-6, 500)
        mu_g = torch.zeros_like(dmu)
        nv.mfs_get_density(ctx, 0, mu_g)
        em_g = nv.mfs_boundary_residual(ctx, problem, mu_g, given, out if problem == "mobility" else given, 64)
        say(f"  GPU solve ({info['iters']} iterations): eps_max {em_g:.6e}")
        assert abs(em_g - em_ref) <= 1e-6
        with pytest.raises(nv.MFSError) as e:
            nv.mfs_get_density(ctx, 1, mu_g)
        assert e.value.code == nv.MFS_ERR_ARG
    finally:
        nv.mfs_destroy(ctx)
