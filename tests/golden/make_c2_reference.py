"""Write tests/golden/c2_reference.npz: FP64 oracle solutions of the P = 1000 workload.

Workload: area fraction 0.5, min gap 1e-2, N_c = 36 on radius 0.7, M_c = 72, contact
threshold 0.2 (workloads.config_geometry(2)); mobility with N(0,1) forces (zero net force)
and torques, resistance with N(0,1) velocities.  Solved by the oracle (Alg. 3 matvec,
unrestarted GMRES) to relative residual 1e-10.  Only oracle/ and workloads/ are used.

Run from the repository root:  python tests/golden/make_c2_reference.py
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.params import MFSParams  # noqa: E402
from oracle.system import System, solve  # noqa: E402
from workloads import config_geometry, mobility_rhs, resistance_rhs  # noqa: E402


def main():
    g = config_geometry(2)
    P = g["centers"].shape[0]
    prm = MFSParams(delta_c=g["delta_c"])
    out = dict(centers=g["centers"], radii=g["radii"], seed=g["seed"])
    for problem in ("mobility", "resistance"):
        given = mobility_rhs(g["seed"], P) if problem == "mobility" else resistance_rhs(g["seed"], P)
        t0 = time.time()
        S = System(g["centers"], g["radii"], g["n_src"], g["n_col"], g["r_src"], problem, prm, progress=True)
        t1 = time.time()
        res, mu, info = solve(S, given, 1e-10, maxit=600,
                              callback=lambda k, r: print(f"  {problem} it {k} resid {r:.3e}", flush=True)
                              if k % 10 == 0 else None)
        print(f"{problem}: pairs {len(S.pairs)} precompute {t1 - t0:.0f}s solve {time.time() - t1:.0f}s "
              f"iters {info['iters']} true resid {info['true_resid']:.2e}", flush=True)
        out[f"{problem}_given"] = given
        out[f"{problem}_out"] = res
        out[f"{problem}_iters"] = info["iters"]
        out[f"{problem}_true_resid"] = info["true_resid"]
        out["pairs"] = S.pairs
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_reference.npz"), **out)


if __name__ == "__main__":
    main()
