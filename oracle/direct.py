"""Brute-force fine-grid MFS solves used only to pin the compressed method (oracle).

These solve the multi-body problem directly with one global least-squares system
on fine point sets, with no one-body preconditioning, no pair corrections and no
compression:

* mobility, "recompleted" form (Sec. 4.1 and Sec. 4.3 generalised to all bodies):
  u = S(x, Y)[(I - L) beta + beta_0], beta_0^(b) = K_b (K_b^T K_b)^{-1} [f; t]^(b),
  rigid velocity ansatz [v; omega]^(b) = -K_b^T beta^(b), and the no-slip
  condition S(X, Y)(I - L) beta + B K^T beta = -S(X, Y) beta_0 at all nodes,
  solved by a truncated-SVD least-squares solve;
* resistance: S(X, Y) beta = B [v; omega], [f; t]^(b) = K_b^T beta^(b).

Bodies in the list may carry any point sets; the pair tests use the pair's fine
sets (Sec. 5) for the near-contact bodies and a fine proxy ring for the others.
"""

from __future__ import annotations

import numpy as np
from scipy.linalg import block_diag

from .geometry import rigid_map, rigid_projector
from .kernel import stokeslet_matrix
from .onebody import apply_pinv, truncated_svd


def direct_solve(bodies, given, problem, mu=1.0, eps=1e-11, strengths=False):
    """bodies: list of (centre, sources (n,2), nodes (m,2)); given: (nb, 3).  Returns (nb, 3), and
    with strengths=True also (Y, sigma): the flow is u(x) = S(x, Y) sigma everywhere outside
    the bodies (mobility: sigma = (I - L) beta + beta_0; resistance: sigma = beta)."""
    Y = np.concatenate([b[1] for b in bodies])
    X = np.concatenate([b[2] for b in bodies])
    K = [rigid_map(b[1], b[0]) for b in bodies]
    B = [rigid_map(b[2], b[0]) for b in bodies]
    S = stokeslet_matrix(X, Y, mu)
    given = np.asarray(given, dtype=np.float64).reshape(len(bodies), 3)
    if problem == "mobility":
        IL = block_diag(*[np.eye(k.shape[0]) - rigid_projector(k) for k in K])
        F = S @ IL + block_diag(*[b @ k.T for b, k in zip(B, K)])
        beta0 = np.concatenate([k @ np.linalg.solve(k.T @ k, given[j]) for j, k in enumerate(K)])
        rhs = -(S @ beta0)
    else:
        F = S
        rhs = np.concatenate([b @ given[j] for j, b in enumerate(B)])
    U, s, Vt = truncated_svd(F, eps)
    beta = apply_pinv(U, s, Vt, rhs)
    out = []
    off = 0
    for k in K:
        n = k.shape[0]
        r = k.T @ beta[off:off + n]
        out.append(-r if problem == "mobility" else r)
        off += n
    if strengths:
        sigma = IL @ beta + beta0 if problem == "mobility" else beta
        return np.array(out), Y, sigma
    return np.array(out)
