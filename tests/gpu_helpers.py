"""Shared helpers of the GPU tests (not collected: no test_ prefix)."""

from __future__ import annotations

import math
import sys

import numpy as np

from oracle.geometry import ring
from oracle.kernel import direct_sum


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def coarse_points(centers, radii, n_src, n_col, r_src):
    """Absolute coarse sources and nodes (oracle construction: equispaced rings from angle 0)."""
    P = centers.shape[0]
    Y = np.concatenate([ring(centers[i], r_src[i] * radii[i], int(n_src[i])) for i in range(P)])
    X = np.concatenate([ring(centers[i], radii[i], int(n_col[i])) for i in range(P)])
    src_off = np.concatenate([[0], np.cumsum(n_src)]).astype(np.int64)
    col_off = np.concatenate([[0], np.cumsum(n_col)]).astype(np.int64)
    return X, Y, src_off, col_off


def oracle_sum_excluding_self(X, Y, sig, src_off, col_off, targets=None, mu=1.0, include_self=False, partners=None):
    """u_t = sum over sources not on the target's disk (or all sources) of S(x_t, y_s) sig_s, and the
    magnitude sum_s (|log r| + 1) |sig_s| / (4 pi mu) that bounds rounding in either precision.
    partners: optional list of sets; sources of those disks are left out as well."""
    P = len(src_off) - 1
    body_of_t = np.repeat(np.arange(P), np.diff(col_off))
    tsel = np.arange(X.shape[0]) if targets is None else np.asarray(targets)
    u = direct_sum(X[tsel], Y, sig, mu)
    mag = np.zeros(len(tsel))
    sabs = np.abs(sig).sum(1)
    blk = max(1, 2_000_000 // max(1, Y.shape[0]))
    for j0 in range(0, len(tsel), blk):
        tt = tsel[j0:j0 + blk]
        d = X[tt][:, None, :] - Y[None, :, :]
        r = np.sqrt((d ** 2).sum(-1))
        mag[j0:j0 + blk] = ((np.abs(np.log(r)) + 1.0) * sabs[None, :]).sum(1) / (4 * math.pi * mu)
    if not include_self:
        for j, t in enumerate(tsel):
            b = body_of_t[t]
            for bb in [b] + (sorted(partners[b]) if partners is not None else []):
                s0, s1 = src_off[bb], src_off[bb + 1]
                u[j] -= direct_sum(X[t:t + 1], Y[s0:s1], sig[s0:s1], mu)[0]
    return u, mag
