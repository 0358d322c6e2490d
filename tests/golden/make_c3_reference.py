"""Write FP64 oracle mobility solutions on the dense-packing generator.

Workload (workloads.config_geometry(3, P=1000)): the generator of the P = 10^4 benchmark
packing (perturbed triangular lattice at area fraction 0.65, pairwise-repulsion relaxation
to min gap 1e-3, Monte-Carlo sweeps, closest pair at gap exactly 1e-3) at P = 1000, which
the oracle solves in tens of minutes, M_c = 72, contact threshold 0.2, and either
* coarse (tests/golden/c3_reference.npz): N_c = 36 sources on radius 0.7, or
* paper (tests/golden/c3p_reference.npz): N_c = 60 sources on the ring-rule radius
  1 - ln(10^12)/60, the paper's coarse discretisation of its P = 10^4 run (Sec. 6.2).
Two right-hand sides (Sec. 6.2 and Fig. 1; Sec. 6.1):
* unit torque on every disk, zero force;
* N(0,1) forces (shifted to zero net force) and torques.
Each is solved by the oracle (Alg. 3 matvec with the direct O(N_s N_t) sum, unrestarted
GMRES, Sec. 4.4 post-processing) to a GMRES residual estimate of 1e-10.  With 60 sources on
the ring-rule radius the one-body pseudoinverse amplifies the top ring modes about 4e10-fold,
and the direct sum's rounding then bounds the true residual near 2e-8 (stored as
*_true_resid); the velocities are still far more accurate than the 1e-5 comparison needs.  Only oracle/ and workloads/
are used; the pair matrices are formed by the oracle's pair_matrices in worker processes
(one pair per task), which changes no arithmetic.

Run from the repository root:  python tests/golden/make_c3_reference.py [coarse|paper]
"""

import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np
from threadpoolctl import threadpool_limits

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.geometry import contacts  # noqa: E402
from oracle.onebody import one_body  # noqa: E402
from oracle.pairs import pair_matrices  # noqa: E402
from oracle.params import MFSParams  # noqa: E402
from oracle.system import System, solve  # noqa: E402
from workloads import config_geometry, mobility_rhs, unit_torques  # noqa: E402

P = 1000
TOL = 1e-10
_W = {}


def _pair(idx):
    i, k = _W["pairs"][idx]
    with threadpool_limits(1):
        return idx, pair_matrices(_W["c"][i], _W["c"][k], _W["ob"], _W["prm"], ob_k=_W["ob"])


def main(kind):
    g = config_geometry(3, P=P)
    prm = MFSParams(delta_c=g["delta_c"])
    assert np.all(g["radii"] == 1.0) and np.all(g["n_src"] == 36)
    n_src, r_src = (60, 1.0 - math.log(1e12) / 60.0) if kind == "paper" else (36, 0.7)
    pairs = contacts(g["centers"], g["radii"], prm.delta_c)
    t0 = time.time()
    _W.update(pairs=pairs, c=g["centers"], prm=prm,
              ob=one_body(1.0, n_src, 72, r_src, prm.mu, "mobility", prm.eps_trunc, prm.eps_ring))
    pd = [None] * len(pairs)
    with mp.get_context("fork").Pool(os.cpu_count() or 1) as pool:
        for n_done, (idx, d) in enumerate(pool.imap_unordered(_pair, range(len(pairs)), chunksize=4)):
            pd[idx] = d
            if n_done % 100 == 0:
                print(f"  pair {n_done}/{len(pairs)}  {time.time() - t0:.0f}s", flush=True)
    S = System(g["centers"], g["radii"], n_src, 72, r_src, "mobility", prm, pair_data=pd)
    assert np.array_equal(S.pairs, pairs)
    print(f"P {P}: {len(pairs)} pairs, precompute {time.time() - t0:.0f}s", flush=True)
    out = dict(P=P, centers=g["centers"], pairs=S.pairs, tol=TOL, n_src=n_src, n_col=72, r_src=r_src)
    for name, given in (("torque", unit_torques(P)), ("random", mobility_rhs(g["seed"], P))):
        t1 = time.time()
        res, mu, info = solve(S, given, TOL, maxit=800,
                              callback=lambda k, r: print(f"  {name} it {k} resid {r:.3e}  {time.time() - t1:.0f}s",
                                                          flush=True) if k % 10 == 0 else None)
        print(f"{name}: solve {time.time() - t1:.0f}s, iters {info['iters']}, true resid {info['true_resid']:.2e}",
              flush=True)
        out[f"{name}_given"] = given
        out[f"{name}_out"] = res
        out[f"{name}_iters"] = info["iters"]
        out[f"{name}_true_resid"] = info["true_resid"]
        out[f"{name}_resid_hist"] = np.asarray(info["resid"])
    name = "c3p_reference.npz" if kind == "paper" else "c3_reference.npz"
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)), name), **out)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "coarse")
