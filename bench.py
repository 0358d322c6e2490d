"""Benchmark: Stokeslet pair-evals/s and time-to-solve of the P = 10^4 mobility problem.

Workload: P = 10000 unit disks at area fraction 0.65 (seeded perturbed triangular
lattice relaxed to a minimum gap of 1e-3, about 0.99 P close pairs), 72 collocation nodes
per disk ("72 vector unknowns per body"), unit torque on every disk, zero forces.  The
coarse discretisation is the paper's for this experiment (Sec. 6.2): 60 Stokeslet sources
on the ring-rule radius 1 - ln(10^12)/60 = 0.5395, GMRES relative-residual tolerance 1e-8
(--discretisation coarse: 36 sources on radius 0.7, tolerance 5e-9, the configuration of
the smaller workloads).  The solution is checked against a plain-FP64 solve of the same
input to relative residual 1e-10 (eq. rel_vel_err).  One step is one
full mobility solve through the C ABI: right-hand side, GMRES on the Alg. 3 operator with
the kernel sum relaxed to FP32 (FP64 accumulation) as the residual falls, FP64 refinement
on the true residual, and post-processing to velocities.  Setup and the pair precompute happen before the
timed region and are reported separately; the plain-FP64 solve of the same input
is run once beside it for the mixed-vs-FP64 comparison.  After the timed region the
relative boundary residual of the mixed solution (eqs. residual_x, residual: the flow
evaluated with each pair's fine sources at 72 points per disk) is reported beside it.

Prints one JSON line.  --gpus N > 1 exits: the benchmark runs on one GPU.

--workload bidisperse replaces the packing by disks of radii 1 and 1.4 (assigned 50/50,
area fraction 0.62, min gap 1e-4; 36/72 and 50/100 coarse points on radius 0.7 a),
default P = 2000, usually with --rhs 8 (unit torques plus seven N(0,1) right-hand sides
with zero net force, solved in lockstep).

--serve runs the serving workload instead: a stream of independent mobility solves
(P ~ U{50..3000}, area fraction U[0.4, 0.65], min gap 10^U[-4,-2], N(0,1) forces and
torques) through the continuous-batching server; first a saturated pass (all requests
queued at once; 16 by default) for solves/s, then a Poisson stream (64 requests) at 0.8 x that rate for the time to
solution (p50, p99).  It prints its own JSON line.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_PAIR = 20          # algorithmic flops of one Stokeslet evaluation applied to a 2-vector
KSUM_T = 2                  # targets per thread of both kernel sums
CELL_ORDER = 31             # order of the cells' moments (the translations' source order)
LOC32_ORDER, LOC64_ORDER = 31, 31   # local expansion orders of the mixed and FP64 kernel sums
LOC32_SEP, LOC64_SEP = 2.0, 3.0     # their separation factors (theta <= 1/2, 1/3)


def flop_ring_expansions(n, terms, merged=False):
    """n evaluations of a disk's ring expansion whose orders sum to terms: three complex Horner
    series, 24 flops per step (p - 1 steps at order p), plus about 66 for zeta, the first terms,
    the log term and the combination (two of them transcendental); merged (the FP32 form): two
    series, one in zeta and one in conj(zeta) that carries the other two, 20 flops per step, plus
    57."""
    if merged:
        return 20 * (terms - n) + 57 * n
    return 24 * (terms - n) + 66 * n


def flop_per_translation(order, src_order=CELL_ORDER):
    """A cell's moments (order src_order) translated into a local expansion of the given order,
    two analytic functions: the moments scaled by Delta^-k (6 flops each), the binomial sums (a
    real times a complex number added, 4 flops per term) and the scaling of the results by
    Delta^-l (6 flops each)."""
    return 2 * (4 * src_order * (order + 1) + 6 * src_order + 6 * (order + 1))


def flop_per_local_evaluation(order):
    """A local expansion at a node: three complex Horner series (L1, L1', L2), 8 flops a step."""
    return 24 * order + 8


def ksum_flops_split(work, mixed):
    """Algorithmic flops of the work a kernel sum counted (mfs_kernel_sum_work), as (FP64, FP32):
    the mixed sum evaluates the near disks' ring expansions in FP32 and everything else (direct
    pairs, translations, local expansions) in FP64."""
    direct, n, terms, m2l, l2p = work
    q = LOC32_ORDER if mixed else LOC64_ORDER
    ring = flop_ring_expansions(n, terms, merged=mixed)
    # the translations take the cells' moments up to the local order
    f64 = direct * FLOP_PER_PAIR + m2l * flop_per_translation(q, q) + l2p * flop_per_local_evaluation(q)
    return (f64, ring) if mixed else (f64 + ring, 0)


def ksum_flops(work, mixed):
    """Algorithmic flops of the work a kernel sum counted."""
    return sum(ksum_flops_split(work, mixed))


def alu_peak_tflops(f64, f32):
    """The VALU peak for a flop mix: the published rates (FP64 78.6, FP32 157.3 TFLOP/s) give
    the shortest time f64 / 78.6 + f32 / 157.3, and the peak is the total over that time."""
    t = f64 / PEAK_FP64_TFLOPS + f32 / PEAK_FP32_TFLOPS
    return (f64 + f32) / t if t > 0 else PEAK_FP64_TFLOPS


def visiting_order(n_col, slot_body):
    """The kernel sums' target order: the nodes of the disks in slot order (mfs_get_clusters)."""
    import numpy as np
    col_off = np.concatenate([[0], np.cumsum(np.asarray(n_col, dtype=np.int64))])
    return np.concatenate([np.arange(col_off[b], col_off[b + 1]) for b in slot_body])


PEAK_FP32_TFLOPS = 157.3    # MI355X published FP32 vector peak (256 CUs, 2.4 GHz)
PEAK_FP64_TFLOPS = 78.6     # MI355X published FP64 vector peak

# HBM traffic of one kernel-sum launch (k_ksum_fmm_mixed, k_ksum_fmm_fp64) on this workload:
# rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE (KiB per dispatch), each scaled by what the counter
# reads for an elementwise kernel that reads and writes 1 GiB.  It holds for the kernel source it
# was measured on, identified by a hash of kernels.hip; None until measured.
KSUM_TRAFFIC = {
    "src_sha256_16": "8a8f34a265271f95",
    "mixed": {"fetch_kib": 101368.0, "fetch_factor": 2.0, "write_kib": 12391.56, "write_factor": 1.0},
    "fp64": {"fetch_kib": 266924.56, "fetch_factor": 2.0, "write_kib": 12391.56, "write_factor": 1.0},
}


def ksum_traffic_bytes(mixed):
    """HBM bytes per kernel-sum launch, or None once the kernels differ from the measured ones."""
    import hashlib
    t = KSUM_TRAFFIC and KSUM_TRAFFIC.get("mixed" if mixed else "fp64")
    if not t:
        return None
    src = open(os.path.join(ROOT, "paper_2606_11273_amd", "csrc", "kernels.hip"), "rb").read()
    if hashlib.sha256(src).hexdigest()[:16] != KSUM_TRAFFIC["src_sha256_16"]:
        return None
    return int((t["fetch_kib"] * t["fetch_factor"] + t["write_kib"] * t["write_factor"]) * 1024)


def rel_rigid_error(out, ref):
    """max_i (|v_i - v_ref,i| + |w_i - w_ref,i|) / max_j (|v_ref,j| + |w_ref,j|) (eq. rel_vel_err)."""
    import numpy as np
    e = np.linalg.norm(out[:, :2] - ref[:, :2], axis=1) + np.abs(out[:, 2] - ref[:, 2])
    s = np.linalg.norm(ref[:, :2], axis=1) + np.abs(ref[:, 2])
    return float(e.max() / s.max())


def cpu_baseline(centers, radii, n_src, n_col, r_src, n_targets, sig_seed=1):
    """The FP64 oracle's direct sum timed on the host cores on a sample of the workload's targets.

    It forks worker processes, so it runs before this process touches the GPU."""
    import numpy as np
    from oracle.geometry import ring
    from oracle.kernel import direct_sum
    P = centers.shape[0]
    Y = np.concatenate([ring(centers[i], r_src[i] * radii[i], int(n_src[i])) for i in range(P)])
    X = np.concatenate([ring(centers[i], radii[i], int(n_col[i])) for i in range(P)])
    rng = np.random.default_rng(sig_seed)
    sig = rng.standard_normal((Y.shape[0], 2))
    tsel = np.sort(rng.choice(X.shape[0], n_targets, replace=False))
    host = os.cpu_count() or 1
    workers = min(16, host)
    t0 = time.perf_counter()
    direct_sum(X[tsel], Y, sig, workers=workers, chunk_elems=2_000_000)
    dt = time.perf_counter() - t0
    evals = n_targets * Y.shape[0]
    return dict(rate=evals / dt, rate_unit="pair-evals/s", cores=workers, host_cores=host, kind="oracle",
                sample=f"{n_targets} of {X.shape[0]} targets x {Y.shape[0]} sources of the same packing, "
                       f"FP64 NumPy direct sum in {workers} single-threaded worker processes "
                       f"({host} host cores), {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", choices=("packed", "bidisperse"), default="packed",
                    help="packed: unit disks at area fraction 0.65, min gap 1e-3 (default P 10000); "
                         "bidisperse: radii 1 and 1.4 (50/50) at area fraction 0.62, min gap 1e-4, 36/50 "
                         "coarse sources (default P 2000)")
    ap.add_argument("--P", type=int, default=None)
    ap.add_argument("--discretisation", choices=("paper", "coarse"), default="paper",
                    help="packed workload: paper = 60 sources on radius 1 - ln(1e12)/60 and 72 nodes per disk "
                         "(Sec. 6.2); coarse = 36 sources on radius 0.7 and 72 nodes")
    ap.add_argument("--tol", type=float, default=None,
                    help="relative residual (default 1e-8 for the paper discretisation, 5e-9 for the coarse "
                         "one, whose velocities at 1e-7 are still ~1e-4 from the converged ones)")
    ap.add_argument("--no-ref", action="store_true",
                    help="skip the FP64 reference solve to relative residual 1e-10")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain-FP64 comparison solve")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-targets", type=int, default=24000,
                    help="targets of the CPU oracle sample (all sources; about 13 s on 16 cores)")
    ap.add_argument("--ksum-reps", type=int, default=5)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB-in, 1 GiB-out elementwise kernel (reference for HBM counters)")
    ap.add_argument("--rhs", type=int, default=1,
                    help="stacked right-hand sides solved in lockstep: #1 unit torques, the others N(0,1) "
                         "forces and torques with zero net force")
    ap.add_argument("--serve", action="store_true", help="run the serving workload (see the module doc)")
    ap.add_argument("--requests", type=int, default=64, help="requests in the Poisson stream (--serve)")
    ap.add_argument("--saturated", type=int, default=16, help="requests in the saturated pass (--serve)")
    ap.add_argument("--slots", type=int, default=4, help="server slots (--serve)")
    ap.add_argument("--no-flow", action="store_true",
                    help="skip the boundary residual of the solution (flow evaluation with the pairs' fine "
                         "sources at --flow-nodes points per disk, after the timed region)")
    ap.add_argument("--flow-nodes", type=int, default=72)
    ap.add_argument("--precompute-only", action="store_true",
                    help="setup and the pair precompute only, then exit (a short program for profiling it)")
    ap.add_argument("--kernel-only", action="store_true",
                    help="set up the workload and run only the dominant kernel (5 launches), then one mixed "
                         "and one FP64 matvec with zero pair matrices (plus --copy-calibration): the short "
                         "program the hardware-counter runs profile")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the hot path runs on one GPU; runs on several GPUs are not implemented "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.serve:
        return run_serving(args)
    # the library prints precompute progress and stage times to stderr with this set
    os.environ.setdefault("MFS_PROFILE", "1")
    import numpy as np
    from workloads import config_geometry, mobility_rhs, unit_torques

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    bidisperse = args.workload == "bidisperse"
    g = config_geometry(5 if bidisperse else 3, P=args.P or (2000 if bidisperse else 10000))
    c, a, ns, nc, rs = g["centers"], g["radii"], g["n_src"], g["n_col"], g["r_src"]
    P = c.shape[0]
    paper = not bidisperse and args.discretisation == "paper"
    if paper:
        # the paper's coarse discretisation of its P = 10^4 run: N_c = 60 on the ring rule, M_c = 72
        ns = np.full(P, 60, dtype=np.int32)
        nc = np.full(P, 72, dtype=np.int32)
        rs = np.full(P, 1.0 - math.log(1e12) / 60.0)
    if args.tol is None:
        args.tol = 1e-8 if paper else 5e-9
    cpu = None
    if not args.no_cpu and not args.kernel_only and not args.precompute_only:
        # the oracle's worker processes are forked before this process touches the GPU
        cpu = cpu_baseline(c, a, ns, nc, rs, args.cpu_targets)
        log(f"cpu baseline {cpu['rate']:.3e} pair-evals/s in {cpu['cores']} processes "
            f"({cpu['host_cores']} host cores)")

    import torch
    from paper_2606_11273_amd import native as nv
    torch.cuda.set_device(0)
    given = unit_torques(P)
    if args.rhs > 1:
        given = np.stack([given] + [mobility_rhs(g["seed"] + r, P) for r in range(1, args.rhs)])
    prm = nv.mfs_default_params()
    prm.delta_c = g["delta_c"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx = nv.mfs_setup(c, a, ns, nc, rs, prm)
    t_setup = time.perf_counter() - t0
    if args.kernel_only:
        _, Ns, Nt, _ = nv.mfs_get_sizes(ctx)
        sig = torch.randn(2 * Ns, dtype=torch.float64, device="cuda")
        u = torch.zeros(2 * Nt, dtype=torch.float64, device="cuda")
        for prec in ("mixed", "fp64"):
            nv.mfs_time_kernel_sum(ctx, prec, sig, u, 2, args.ksum_reps)
        # two whole matvecs (mixed, then FP64) so that counters also cover the pair-correction
        # kernels; the pair matrices are zeros of the right shapes (same memory traffic)
        sizes = [2 * int(ns[i] + ns[k]) for i, k in nv.mfs_get_pairs(ctx)]
        nv.mfs_set_pair_matrices(ctx, "mobility", [np.zeros((m, m)) for m in sizes], [np.zeros((6, m)) for m in sizes])
        mu = torch.randn(2 * Nt, dtype=torch.float64, device="cuda")
        w = torch.zeros_like(mu)
        for prec in ("mixed", "fp64"):
            nv.mfs_apply(ctx, "mobility", prec, mu, w)
        if args.copy_calibration:
            # an elementwise kernel that reads 1 GiB and writes 1 GiB (a same-dtype copy_ could
            # go to the DMA engines, which the shader counters do not see)
            buf = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
            out = torch.empty_like(buf)
            torch.neg(buf, out=out)
        torch.cuda.synchronize()
        nv.mfs_destroy(ctx)
        print(json.dumps({"kernel_only": True, "launches": args.ksum_reps, "copy_bytes": (1 << 30) if
                          args.copy_calibration else 0}), flush=True)
        return
    if not args.no_flow and not args.precompute_only:
        nv.mfs_keep_fine_factors(ctx, True)
    t0 = time.perf_counter()
    n_pairs = nv.mfs_precompute_pairs(ctx, "mobility")
    torch.cuda.synchronize()
    t_pre = time.perf_counter() - t0
    _, Ns, Nt, _ = nv.mfs_get_sizes(ctx)
    log(f"setup {t_setup:.2f}s  precompute {n_pairs} pairs {t_pre:.2f}s  Ns {Ns} Nt {Nt}")
    if args.precompute_only:
        nv.mfs_destroy(ctx)
        print(json.dumps({"precompute_only": True, "P": P, "pairs": n_pairs, "precompute_s": round(t_pre, 3),
                          "setup_s": round(t_setup, 3)}), flush=True)
        return

    # the kernel sums in the matvec's launch configuration (skip own disk and partners): HIP events
    # on the context's stream around the sum kernel alone (mfs_time_kernel_sum), work as counted
    stream = torch.cuda.current_stream()
    sig = torch.randn(2 * Ns, dtype=torch.float64, device="cuda")
    u = torch.zeros(2 * Nt, dtype=torch.float64, device="cuda")
    ks, krec, kwork = {}, {}, {}
    for prec in ("mixed", "fp64"):
        nv.mfs_time_kernel_sum(ctx, prec, sig, u, 2, 1)
        nv.mfs_kernel_sum_work(ctx, reset=True)
        krec[prec], ks[prec] = nv.mfs_time_kernel_sum(ctx, prec, sig, u, 2, args.ksum_reps)
        kwork[prec] = tuple(w // args.ksum_reps for w in nv.mfs_kernel_sum_work(ctx, reset=True))

    # plain FP64 solve of the same input (comparison)
    out64 = None
    info64 = {}
    t_fp64 = None
    if not args.no_fp64:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out64, info64 = nv.mfs_gmres_solve(ctx, "mobility", "fp64", given, args.tol, 1000)
        t_fp64 = time.perf_counter() - t0
        log(f"fp64 solve {t_fp64:.2f}s iters {info64['iters']} resid {info64['rel_resid']:.2e}")

    for _ in range(args.warmup):
        nv.mfs_gmres_solve(ctx, "mobility", "mixed", given, args.tol, 1000)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    infos = []
    e0.record(stream)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out32, info32 = nv.mfs_gmres_solve(ctx, "mobility", "mixed", given, args.tol, 1000)
        infos.append(info32)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    log(f"mixed solve {ms:.1f} ms/solve (wall {wall / args.steps * 1e3:.1f}) iters {infos[-1]['iters']} "
        f"outer {infos[-1]['outer']} resid {infos[-1]['rel_resid']:.2e}")
    last = infos[-1]
    solve_work = {k: last[k] for k in ("dense_pairs", "direct_pairs", "ring_expansions", "expansion_terms",
                                       "local_translations", "local_evaluations")}
    value = ms / 1e3

    if args.copy_calibration:
        buf = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        out = torch.empty_like(buf)
        torch.neg(buf, out=out)
        torch.cuda.synchronize()

    # roofline of the dominant kernel: the kernel sum the timed solve applied most (mixed or FP64;
    # one launch = one matvec's sum without each disk's own sources and its contact partners).
    # Its algorithmic flops are the work the kernel counted itself (ksum_flops); dense_pairs is
    # the count of the plain direct sum a launch stands for, which the kernel does not evaluate.
    pr = nv.mfs_get_pairs(ctx)
    skipped = ns.astype(np.int64).copy()
    np.add.at(skipped, pr[:, 0], ns[pr[:, 1]])
    np.add.at(skipped, pr[:, 1], ns[pr[:, 0]])
    dense_launch = int(np.sum(nc.astype(np.int64) * (Ns - skipped)))
    dom = "mixed" if last["matvecs_mixed"] >= last["matvecs_fp64"] else "fp64"
    kern = {}
    for prec in ("mixed", "fp64"):
        f64, f32 = ksum_flops_split(kwork[prec], prec == "mixed")
        fl = f64 + f32
        sec = ks[prec] * 1e-3
        d, n, terms, m2l, l2p = kwork[prec]
        peak = alu_peak_tflops(f64, f32)
        kern[prec] = dict(ms_per_launch=round(ks[prec], 4), ms_records=round(krec[prec], 4), flops_per_launch=fl,
                          flops_fp64=f64, flops_fp32=f32, peak_tflops=round(peak, 2),
                          tflops=round(fl / sec / 1e12, 2), frac_valu=round(fl / sec / 1e12 / peak, 4),
                          direct_pairs=d, ring_expansions=n, mean_ring_order=round(terms / max(n, 1), 2),
                          local_translations=m2l, local_evaluations=l2p,
                          dense_equivalent_pairs_per_s=round(dense_launch / sec, 1))
        log(f"kernel sum {prec}: {ks[prec]:.3f} ms per launch (+{krec[prec]:.3f} ms packing and records), "
            f"{fl / sec / 1e12:.2f} TFLOP/s; work {kwork[prec]}")
    kd = kern[dom]
    roofline = dict(bound="alu", achieved=kd["tflops"], peak=kd["peak_tflops"], unit="TFLOP/s",
                    frac=kd["frac_valu"], traffic=ksum_traffic_bytes(dom == "mixed"),
                    kernel=f"k_ksum_fmm_{dom} ({dom} kernel sum: per wave of "
                           "128 nodes, cell translations into an FP64 local expansion and near disks from their ring "
                           f"expansions{' in FP32' if dom == 'mixed' else ''})",
                    peak_note="the kernel's own flop mix at the published vector peaks: (FP64 + FP32 flops) / "
                              "(FP64 flops / 78.6 + FP32 flops / 157.3 TFLOP/s); the FP32 flops are the near disks' "
                              "ring expansions",
                    dense_pairs_per_launch=dense_launch, kernels=kern)

    # stacked matvec: one T mu on args.rhs vectors at once, per vector (HIP events)
    stacked = None
    if args.rhs > 1:
        mu = torch.randn(args.rhs * 2 * Nt, dtype=torch.float64, device="cuda")
        w = torch.zeros_like(mu)
        stacked = {}
        for prec in ("mixed", "fp64"):
            nv.mfs_apply(ctx, "mobility", prec, mu, w, n_rhs=args.rhs)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            nv.mfs_apply(ctx, "mobility", prec, mu, w, n_rhs=args.rhs)
            e1.record(stream)
            torch.cuda.synchronize()
            stacked[f"{prec}_ms_per_vector"] = round(e0.elapsed_time(e1) / args.rhs, 2)

    # accuracy of the mixed solution: relative boundary residual (eqs. residual_x, residual) of the
    # first right-hand side, the flow evaluated with each pair's fine sources near contacts
    flow = None
    if not args.no_flow:
        mu0 = torch.zeros(2 * Nt, dtype=torch.float64, device="cuda")
        nv.mfs_get_density(ctx, 0, mu0)
        out_first = out32.reshape(-1, P, 3)[0]
        given_first = given.reshape(-1, P, 3)[0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        em = nv.mfs_boundary_residual(ctx, "mobility", mu0, given_first, out_first, args.flow_nodes)
        t_flow = time.perf_counter() - t0
        flow = {"eps_max": em, "nodes_per_disk": args.flow_nodes, "points": P * args.flow_nodes,
                "seconds": round(t_flow, 3)}
        log(f"boundary residual {em:.3e} at {args.flow_nodes} nodes per disk, {t_flow:.2f}s")

    err = None
    if out64 is not None:
        err = max(rel_rigid_error(a32, a64) for a32, a64 in zip(out32.reshape(-1, P, 3), out64.reshape(-1, P, 3)))
    # accuracy of both forms against a plain-FP64 solve of the same input to relative residual 1e-10
    ref_err = None
    if not args.no_ref:
        t0 = time.perf_counter()
        outr, infor = nv.mfs_gmres_solve(ctx, "mobility", "fp64", given, 1e-10, 1000, allow_noconv=True)
        ref_err = {"mixed": max(rel_rigid_error(x, y) for x, y in zip(out32.reshape(-1, P, 3), outr.reshape(-1, P, 3))),
                   "fp64": (max(rel_rigid_error(x, y) for x, y in zip(out64.reshape(-1, P, 3), outr.reshape(-1, P, 3)))
                            if out64 is not None else None),
                   "reference_iters": infor["iters"], "reference_resid": infor["rel_resid"]}
        log(f"reference FP64 solve to 1e-10: {infor['iters']} iterations, {time.perf_counter() - t0:.1f}s; "
            f"max E mixed {ref_err['mixed']:.2e} fp64 {ref_err['fp64']}")

    line = {
        "metric": "Stokeslet pair-evals/s + time-to-solve P=10k phi=0.65 at 1e-5 (mixed vs FP64)",
        "value": round(value, 4),
        "unit": "s (time to solve, mixed form)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"mobility solve, P={P} "
                               + ("disks of radii 1 and 1.4 (50/50), area fraction 0.62, min gap 1e-4, "
                                  f"{n_pairs} close pairs, N_c/M_c 36/72 and 50/100, R_c=0.7a, "
                                  if bidisperse else
                                  f"unit disks, area fraction 0.65, min gap 1e-3, {n_pairs} close pairs, "
                                  + ("N_c=60 M_c=72 R_c=1-ln(1e12)/60 (the paper's), " if paper else
                                     "N_c=36 M_c=72 R_c=0.7, "))
                               + ("unit torques" if args.rhs == 1 else
                                  f"{args.rhs} right-hand sides in lockstep (unit torques + N(0,1))")
                               + f", GMRES tol {args.tol:g}",
                   "P": P, "n_pairs": n_pairs, "unknowns": 2 * Nt, "rhs": args.rhs,
                   "n_src": int(ns[0]) if not bidisperse else "36/50", "n_col": int(nc[0]) if not bidisperse else "72/100",
                   "tol": args.tol},
        "time_to_solve_s": {"mixed": round(ms / 1e3, 3), "fp64": round(t_fp64, 3) if t_fp64 else None},
        "speedup_mixed_vs_fp64": round(t_fp64 / (ms / 1e3), 2) if t_fp64 else None,
        "max_rel_velocity_diff_mixed_vs_fp64": err,
        "max_rel_velocity_error_vs_fp64_1e-10": ref_err,
        "iterations": {"mixed_inner": infos[-1]["iters"], "mixed_outer": infos[-1]["outer"],
                       "fp64": info64.get("iters")},
        "paper_context": ("the paper's P=10^4 area-fraction-0.65 solve (Sec. 6.2): 47 GMRES iterations to 1e-7, 36 s "
                          "on 96 AMD Genoa cores with an FMM far field, FP64 MATLAB; its own packing"),
        "rel_resid": {"mixed": infos[-1]["rel_resid"], "fp64": info64.get("rel_resid")},
        "kernel_sum_work_per_solve": solve_work,
        "setup_s": round(t_setup, 3),
        "precompute_s": round(t_pre, 2),
        "stacked_matvec": stacked,
        "boundary_residual": flow,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if cpu is not None:
        # the oracle's time to solve in the metric's unit, extrapolated from its measured direct-sum
        # rate: one kernel sum per GMRES iteration over the dense (target, source) pairs a launch
        # stands for; its one-body, pair and orthogonalisation steps and its precompute are left
        # out, so this is a lower bound
        its = infos[-1]["iters"]
        cpu = dict(value=round(its * dense_launch / cpu["rate"], 1),
                   unit="s (oracle time to solve: iterations x dense pairs per kernel sum / oracle rate; lower bound)",
                   iterations=its, dense_pairs_per_kernel_sum=dense_launch, **cpu)
        line["cpu_baseline"] = cpu
    nv.mfs_destroy(ctx)
    print(json.dumps(line), flush=True)


def run_serving(args):
    import numpy as np
    import torch
    from paper_2606_11273_amd import native as nv
    from workloads import poisson_arrivals, serving_request

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    tol = 1e-7
    reqs = [serving_request(k) for k in range(args.saturated + args.requests)]
    srv = nv.mfs_server_create(0, args.slots)

    def submit(r):
        return nv.mfs_server_submit(srv, r["centers"], r["radii"], r["n_src"], r["n_col"], r["r_src"], "mobility",
                                    "mixed", r["given"], tol, 500)

    try:
        warm = serving_request(10**6, P_lo=50, P_hi=60)
        nv.mfs_server_wait(srv, submit(warm), warm["P"])
        # saturated pass: every request queued at once
        sat = reqs[:args.saturated]
        t0 = time.perf_counter()
        pending = {submit(r): r for r in sat}
        while pending:
            for t in list(pending):
                r = pending[t]
                try:
                    nv.mfs_server_wait(srv, t, r["P"], timeout_ms=0)
                except nv.MFSError as e:
                    if e.code == nv.MFS_ERR_STATE:
                        continue
                    raise
                del pending[t]
                log(f"saturated: request P={r['P']} done at {time.perf_counter() - t0:.1f} s")
            time.sleep(0.05)
        sat_rate = len(sat) / (time.perf_counter() - t0)
        # Poisson stream at 0.8 x the saturated rate: submit at the arrival times, collect
        # completions as they happen
        stream = reqs[args.saturated:]
        rate = 0.8 * sat_rate
        arrive = poisson_arrivals(len(stream), rate)
        t0 = time.perf_counter()
        pending = {}
        res = []
        nxt = 0
        while nxt < len(stream) or pending:
            now = time.perf_counter() - t0
            while nxt < len(stream) and arrive[nxt] <= now:
                r = stream[nxt]
                pending[submit(r)] = r
                log(f"stream: submitted P={r['P']} at {now:.1f} s ({len(pending)} in the server)")
                nxt += 1
            for t in list(pending):
                r = pending[t]
                try:
                    out, info = nv.mfs_server_wait(srv, t, r["P"], timeout_ms=0)
                except nv.MFSError as e:
                    if e.code == nv.MFS_ERR_STATE:
                        continue
                    raise
                del pending[t]
                res.append(info)
                log(f"stream: P={r['P']} done at {time.perf_counter() - t0:.1f} s: total {info['ms_total'] / 1e3:.1f} s "
                    f"(queue {info['ms_queue'] / 1e3:.1f}, precompute {info['ms_precompute'] / 1e3:.1f}, "
                    f"iters {info['iters']})")
            time.sleep(0.05)
        wall = time.perf_counter() - t0
    finally:
        nv.mfs_server_destroy(srv)
    tot = np.array([i["ms_total"] for i in res]) / 1e3
    line = {
        "metric": "serving: solves/s and time to solution (continuous batching)",
        "value": round(len(stream) / wall, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{len(stream)} Poisson-arrival mobility solves, P~U[50,3000], area fraction "
                               f"U[0.4,0.65], min gap 10^U[-4,-2], N(0,1) forces/torques, tol {tol:g}, mixed",
                   "slots": args.slots, "arrival_rate_per_s": round(rate, 4)},
        "saturated_solves_per_s": round(sat_rate, 4),
        "time_to_solution_s": {"p50": round(float(np.percentile(tot, 50)), 3),
                               "p99": round(float(np.percentile(tot, 99)), 3),
                               "mean": round(float(tot.mean()), 3)},
        "service_s_mean": round(float(np.mean([i["ms_service"] for i in res])) / 1e3, 3),
        "precompute_s_mean": round(float(np.mean([i["ms_precompute"] for i in res])) / 1e3, 3),
        "P_mean": round(float(np.mean([r["P"] for r in stream])), 1),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
