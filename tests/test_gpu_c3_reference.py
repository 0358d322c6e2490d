"""GPU solves of the dense-packing workload against stored FP64 oracle solutions.

tests/golden/c3_reference.npz is written by tests/golden/make_c3_reference.py, which calls
only oracle/ and workloads/: the generator of the P = 10^4 benchmark packing (area fraction
0.65, perturbed lattice relaxed to min gap 1e-3, Monte-Carlo sweeps, closest pair at gap
exactly 1e-3) at P = 1000, N_c = 36 on radius 0.7, M_c = 72, contact threshold 0.2, with unit
torques (Fig. 1) and with N(0,1) forces (zero net force) and torques (Sec. 6.1), each solved
by the oracle to relative residual 1e-10; and the same with the paper's coarse discretisation
of its P = 10^4 run (tests/golden/c3p_reference.npz: N_c = 60 on the ring-rule radius
1 - ln(10^12)/60).  The GPU runs its own precompute (device SVDs) and GMRES, plain FP64 and
relaxed mixed, to 5e-9 (the mixed form with N(0,1) forces to 1e-9; 1e-8 and 3e-8 with 60-source rings).  Bar: max_i E^(i) <= 1e-5
(eq. rel_vel_err with the max-speed normalisation).
"""

import math
import os

import numpy as np
import pytest

from oracle.system import rel_rigid_error
from workloads import config_geometry, mobility_rhs, unit_torques
from tests.gpu_helpers import say

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
CASES = {"coarse": (os.path.join(GOLDEN, "c3_reference.npz"), 36, 0.7),
         "paper": (os.path.join(GOLDEN, "c3p_reference.npz"), 60, 1.0 - math.log(1e12) / 60.0)}

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["coarse", "paper"])
def test_dense_packing_solves_match_stored_oracle_solutions(kind):
    from paper_2606_11273_amd import native as nv
    path, n_src, r_src = CASES[kind]
    if not os.path.exists(path):
        pytest.skip(f"run tests/golden/make_c3_reference.py {kind} first")
    ref = np.load(path)
    P = int(ref["P"])
    if "n_src" in ref:
        assert int(ref["n_src"]) == n_src and float(ref["r_src"]) == r_src
    g = config_geometry(3, P=P)
    assert np.array_equal(ref["centers"], g["centers"])
    rhs = {"torque": unit_torques(P), "random": mobility_rhs(g["seed"], P)}
    for name, given in rhs.items():
        assert np.array_equal(ref[f"{name}_given"], given)
    prm = nv.mfs_default_params()
    prm.delta_c = g["delta_c"]
    ctx = nv.mfs_setup(g["centers"], g["radii"], np.full(P, n_src), np.full(P, 72), np.full(P, r_src), prm)
    try:
        assert np.array_equal(nv.mfs_get_pairs(ctx), ref["pairs"].astype(np.int32))
        say(f"dense packing P={P}, {kind} discretisation: precompute {nv.mfs_precompute_pairs(ctx, 'mobility')} pairs")
        for name, given in rhs.items():
            for prec in ("fp64", "mixed"):
                # the benchmark's tolerance for each discretisation (5e-9 and 1e-8), except the
                # mixed form with N(0,1) forces on 36-source rings: at 5e-9 its true residual
                # carried the FP32 noise into slowly converging directions and its velocities
                # were 1.1e-5 from the oracle's (FP64 at the same residual: 3.8e-7).  With 60
                # sources on the ring-rule radius FP64 rounding alone holds the true residual
                # between 6e-9 and 1.1e-8 with unit torques (it moves with the rounding order of
                # equivalent forms of the operator) and near 1.6e-8 with N(0,1) forces (the
                # one-body map amplifies the ring's top modes 4e10-fold; the oracle's own true
                # residual is about 2e-8), so these solves stop at 2e-8 and 3e-8
                if kind == "paper":
                    tol = 2e-8 if name == "torque" else 3e-8
                else:
                    tol = 1e-9 if (prec, name) == ("mixed", "random") else 5e-9
                out, info = nv.mfs_gmres_solve(ctx, "mobility", prec, given, tol, 1000)
                E = rel_rigid_error(out, ref[f"{name}_out"]).max()
                say(f"  {name} {prec} tol {tol:g}: iters {info['iters']} (oracle {int(ref[f'{name}_iters'])} to "
                    f"1e-10), outer {info['outer']}, resid {info['rel_resid']:.2e}, max E {E:.2e}")
                assert info["rel_resid"] <= tol
                assert E <= 1e-5
    finally:
        nv.mfs_destroy(ctx)
