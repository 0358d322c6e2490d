"""Write tests/golden/c2_reference.npz: FP64 oracle solutions of the area-fraction-0.5 workload.

Workload (workloads.config_geometry(2, P)): perturbed triangular lattice at area fraction 0.5
relaxed to min gap 1e-2, N_c = 36 on radius 0.7, M_c = 72, contact threshold 0.2.
* mobility, P = 1000: N(0,1) forces (zero net force) and torques;
* resistance, P = 100: N(0,1) velocities.  At P = 1000 the resistance GMRES does not
  converge within 1000 iterations (relative residual 3.5e-3; lubrication forces between
  the ~370 close pairs make the system far harder than the mobility one), so the stored
  resistance case is the same generator at P = 100 (239 iterations to 1e-10).
Both are solved by the oracle (Alg. 3 matvec, unrestarted GMRES) to relative residual
1e-10.  Only oracle/ and workloads/ are used.

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

SIZES = {"mobility": 1000, "resistance": 100}


def main():
    out = {}
    for problem, P in SIZES.items():
        g = config_geometry(2, P=P)
        prm = MFSParams(delta_c=g["delta_c"])
        given = mobility_rhs(g["seed"], P) if problem == "mobility" else resistance_rhs(g["seed"], P)
        t0 = time.time()
        S = System(g["centers"], g["radii"], g["n_src"], g["n_col"], g["r_src"], problem, prm, progress=True)
        t1 = time.time()
        res, mu, info = solve(S, given, 1e-10, maxit=800,
                              callback=lambda k, r: print(f"  {problem} it {k} resid {r:.3e}", flush=True)
                              if k % 10 == 0 else None)
        print(f"{problem}: P {P}, pairs {len(S.pairs)}, precompute {t1 - t0:.0f}s, solve {time.time() - t1:.0f}s, "
              f"iters {info['iters']}, true resid {info['true_resid']:.2e}", flush=True)
        out[f"{problem}_P"] = P
        out[f"{problem}_centers"] = g["centers"]
        out[f"{problem}_pairs"] = S.pairs
        out[f"{problem}_given"] = given
        out[f"{problem}_out"] = res
        out[f"{problem}_iters"] = info["iters"]
        out[f"{problem}_true_resid"] = info["true_resid"]
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_reference.npz"), **out)


if __name__ == "__main__":
    main()
