"""The serving layer (mfs_server_*): continuous batching of independent solves.

* Each request's result is the same alone and in a mix: a stream of requests of
  different sizes runs through a 3-slot server concurrently and then one at a
  time; the outputs agree to 1e-12 of max |v| + |omega| (the arithmetic of a
  request does not depend on the others, so they are expected to be identical).
* Admission by device-memory footprint: with a budget of 1.5 footprints (one request
  submitted four times), no two requests run together even with 3 slots; a request
  larger than the whole budget is refused.
* Two small requests agree with the FP64 oracle (eq. rel_vel_err <= 1e-5).
Requests come from the serving workload generator (area fraction U[0.4, 0.65], min
gap 10^U[-4,-2], N(0,1) forces and torques with zero net force), with P reduced to
50-150 disks so that the test runs in seconds.
"""

import time

import numpy as np
import pytest

from oracle.params import MFSParams
from oracle.system import System, rel_rigid_error, solve
from workloads import serving_request
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

TOL = 1e-9


def _submit(nv, srv, r, precision="mixed"):
    return nv.mfs_server_submit(srv, r["centers"], r["radii"], r["n_src"], r["n_col"], r["r_src"], "mobility",
                                precision, r["given"], TOL, 300)


def test_server_same_result_alone_and_in_mix():
    from paper_2606_11273_amd import native as nv
    reqs = [serving_request(k, P_lo=50, P_hi=150) for k in range(6)]
    precs = ["mixed", "fp64", "mixed", "mixed", "fp64", "mixed"]
    say("server mix of", [r["P"] for r in reqs])
    srv = nv.mfs_server_create(0, 3)
    try:
        tickets = [_submit(nv, srv, r, p) for r, p in zip(reqs, precs)]
        mixed = [nv.mfs_server_wait(srv, t, r["P"]) for t, r in zip(tickets, reqs)]
    finally:
        nv.mfs_server_destroy(srv)
    overlap = sum(1 for i in range(6) for j in range(i) if mixed[i][1]["ms_queue"] < mixed[j][1]["ms_total"])
    say(f"  in the mix: max total {max(m[1]['ms_total'] for m in mixed):.0f} ms, overlapping pairs {overlap}")
    srv = nv.mfs_server_create(0, 1)
    try:
        for r, p, (out_mix, info_mix) in zip(reqs, precs, mixed):
            out, info = nv.mfs_server_wait(srv, _submit(nv, srv, r, p), r["P"])
            d = rel_rigid_error(out, out_mix).max()
            say(f"  P {r['P']} {p}: iters {info['iters']} resid {info['rel_resid']:.2e}, alone vs mix {d:.1e}"
                f"{' (bitwise equal)' if np.array_equal(out, out_mix) else ''}")
            assert info["rel_resid"] <= TOL and info_mix["rel_resid"] <= TOL
            assert d <= 1e-12
    finally:
        nv.mfs_server_destroy(srv)
    assert overlap > 0   # the three slots did run requests together


def test_server_admits_by_footprint():
    from paper_2606_11273_amd import native as nv
    # one request submitted four times: a budget of 1.5 footprints holds exactly one at a time
    r0 = serving_request(10, P_lo=100, P_hi=100)
    reqs = [r0] * 4
    probe = nv.mfs_server_create(1 << 40, 1)
    try:
        fp = [nv.mfs_server_footprint(probe, r0["centers"], r0["radii"], r0["n_src"], r0["n_col"], r0["r_src"],
                                      "mobility", "mixed", r0["given"], TOL, 300)] * 4
    finally:
        nv.mfs_server_destroy(probe)
    budget = fp[0] + fp[0] // 2
    say("server footprints (MB)", [round(f / 2**20) for f in fp], "budget", budget >> 20)
    srv = nv.mfs_server_create(budget, 3)
    try:
        t_sub = []
        tickets = []
        for r in reqs:
            t_sub.append(time.perf_counter())
            tickets.append(_submit(nv, srv, r))
        res = [nv.mfs_server_wait(srv, t, r["P"])[1] for t, r in zip(tickets, reqs)]
        bad = np.array([[0.0, 0.0], [1.5, 0.0]])
        with pytest.raises(nv.MFSError) as e:
            nv.mfs_server_submit(srv, bad, 1.0, 36, 72, 0.7, "mobility", "mixed", np.zeros((2, 3)), TOL)
        assert e.value.code == nv.MFS_ERR_GEOMETRY
        with pytest.raises(nv.MFSError) as e:
            nv.mfs_server_wait(srv, 10**9, 1)
        assert e.value.code == nv.MFS_ERR_ARG
    finally:
        nv.mfs_server_destroy(srv)
    # a request larger than the whole budget is refused at submission
    tiny = nv.mfs_server_create(min(fp) // 2, 1)
    try:
        with pytest.raises(nv.MFSError) as e:
            _submit(nv, tiny, reqs[0])
        assert e.value.code == nv.MFS_ERR_ARG and "budget" in str(e.value)
    finally:
        nv.mfs_server_destroy(tiny)
    spans = sorted((t0 + i["ms_queue"] / 1e3, t0 + i["ms_total"] / 1e3) for t0, i in zip(t_sub, res))
    for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
        assert b0 >= a1 - 2e-3, "two requests ran together beyond the budget"


def test_server_small_requests_match_oracle():
    from paper_2606_11273_amd import native as nv
    reqs = [serving_request(k, P_lo=50, P_hi=70) for k in (30, 31)]
    srv = nv.mfs_server_create(0, 2)
    try:
        tickets = [_submit(nv, srv, r) for r in reqs]
        outs = [nv.mfs_server_wait(srv, t, r["P"]) for t, r in zip(tickets, reqs)]
    finally:
        nv.mfs_server_destroy(srv)
    for r, (out, info) in zip(reqs, outs):
        S = System(r["centers"], r["radii"], 36, 72, 0.7, "mobility", MFSParams(delta_c=0.2))
        ref, _, rinfo = solve(S, r["given"], TOL)
        E = rel_rigid_error(out, ref).max()
        say(f"  P {r['P']} gap {r['g_min']:.1e}: server iters {info['iters']}, oracle {rinfo['iters']}, max E {E:.2e}")
        assert E <= 1e-5
