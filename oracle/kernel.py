"""The 2D Stokeslet and plain direct sums (oracle).

eq. stokeslet2d (Sec. 3): S(x, y) = 1/(4 pi mu) [ -log|x - y| I + (x - y)(x - y)^T / |x - y|^2 ].
eq. stokes_sum / eq. stokes_operator: u(x) = sum over sources of S(x, y_j) lambda_j.

2-vectors are stacked per point, (x, y) interleaved (a reading of the paper): row 2m + a of
S(X, Y) is component a at target m, column 2n + b is component b of source n.
"""

from __future__ import annotations

import math
import multiprocessing as mp
import os
import sys

import numpy as np
from threadpoolctl import threadpool_limits


def stokeslet_blocks(x, y, mu=1.0):
    """All 2x2 blocks S(x_m, y_n): array (M, N, 2, 2).  Coincident points are not allowed."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 2)
    y = np.asarray(y, dtype=np.float64).reshape(-1, 2)
    d = x[:, None, :] - y[None, :, :]
    r2 = d[..., 0] ** 2 + d[..., 1] ** 2
    logr = 0.5 * np.log(r2)
    out = d[..., :, None] * d[..., None, :] / r2[..., None, None]
    out[..., 0, 0] -= logr
    out[..., 1, 1] -= logr
    return out / (4.0 * math.pi * mu)


def stokeslet_matrix(x, y, mu=1.0):
    """Dense (2M, 2N) matrix S(X, Y) in the interleaved layout."""
    b = stokeslet_blocks(x, y, mu)
    M, N = b.shape[0], b.shape[1]
    return b.transpose(0, 2, 1, 3).reshape(2 * M, 2 * N)


def _sum_chunk(x, y, sig, mu):
    d0 = x[:, 0:1] - y[None, :, 0]
    d1 = x[:, 1:2] - y[None, :, 1]
    r2 = d0 * d0 + d1 * d1
    logr = 0.5 * np.log(r2)
    dot = (d0 * sig[None, :, 0] + d1 * sig[None, :, 1]) / r2
    ux = -(logr @ sig[:, 0]) + np.sum(dot * d0, axis=1)
    uy = -(logr @ sig[:, 1]) + np.sum(dot * d1, axis=1)
    return np.stack([ux, uy], axis=1) / (4.0 * math.pi * mu)


_SHARED = {}


def _gpu_initialised():
    """True once this process has initialised a GPU through torch.

    A process that has initialised the GPU runtime must not fork workers: the children
    inherit device and profiler state they cannot use, and fail when the pool shuts down.
    """
    torch = sys.modules.get("torch")
    if torch is None:
        return False
    try:
        return bool(torch.cuda.is_initialized())
    except Exception:
        return False


def _worker(bounds):
    lo, hi = bounds
    s = _SHARED
    # one thread per worker process: the pool already uses the cores
    with threadpool_limits(1):
        return lo, _sum_chunk(s["x"][lo:hi], s["y"], s["sig"], s["mu"])


def direct_sum(x, y, sig, mu=1.0, workers=None, chunk_elems=4_000_000):
    """u_m = sum_n S(x_m, y_n) sig_n for all targets (eq. stokes_sum), plain O(M N).

    x: (M, 2) targets, y: (N, 2) sources, sig: (N, 2) strengths -> (M, 2).
    Targets are split into blocks; large problems spread the blocks over
    forked worker processes (one block of targets each, no reordering of the sum
    over sources within a target).  In a process that has initialised the GPU the sum
    runs in this process only (workers=None), and workers > 1 is refused.
    """
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 2)
    y = np.ascontiguousarray(y, dtype=np.float64).reshape(-1, 2)
    sig = np.ascontiguousarray(sig, dtype=np.float64).reshape(-1, 2)
    M, N = x.shape[0], y.shape[0]
    out = np.empty((M, 2))
    if M == 0:
        return out
    step = max(1, chunk_elems // max(N, 1))
    bounds = [(lo, min(M, lo + step)) for lo in range(0, M, step)]
    gpu = _gpu_initialised()
    if workers is None:
        # at most 16 processes: hosts that share their cores between jobs give each one that many
        workers = min(len(bounds), os.cpu_count() or 1, 16) if M * N > 5e8 and not gpu else 1
    elif workers > 1 and gpu:
        raise RuntimeError("direct_sum: no worker processes are forked from a process that has "
                           "initialised the GPU (pass workers=1 or None)")
    if workers <= 1 or len(bounds) == 1:
        for lo, hi in bounds:
            out[lo:hi] = _sum_chunk(x[lo:hi], y, sig, mu)
        return out
    _SHARED.update(x=x, y=y, sig=sig, mu=mu)
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        for lo, part in pool.imap_unordered(_worker, bounds):
            out[lo:lo + part.shape[0]] = part
    _SHARED.clear()
    return out
