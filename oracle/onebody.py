"""One-body bases (oracle).

Resistance (Sec. 3.1): the self block P = S(X, Y) of a disk is factorised by the
SVD P = U Sigma V^T and applied as lambda_bar = V Sigma^+ (U^T mu) (eq. howG+),
where Sigma^+ keeps 1/sigma_j only for sigma_j > sigma_1 eps_trunc.

Mobility (Sec. 4.1): with K the rigid map at the sources, B at the nodes and
L = K (K^T K)^{-1} K^T, the one-body matrix is S_L = P (I - L) + B K^T (eq. SL) and
lambda_bar = S_L^+ mu, applied the same way.  Rigid velocities follow the ansatz
[v; omega] = -K^T lambda_bar (eq. rbm_ansatz).

All disks with the same (radius, N_c, M_c, R_c) share these matrices; they are
built in body-relative coordinates.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .geometry import ring, rigid_map, rigid_projector, ring_radius
from .kernel import stokeslet_matrix


def truncated_svd(M, eps):
    """Thin SVD with singular values <= sigma_1 * eps dropped (eq. howG+)."""
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    keep = s > s[0] * eps
    return U[:, keep], s[keep], Vt[keep, :]


def apply_pinv(U, s, Vt, rhs):
    """V Sigma^+ (U^T rhs), applied right to left (eq. howG+)."""
    return Vt.T @ ((U.T @ rhs) / (s[:, None] if rhs.ndim == 2 else s))


@dataclass
class OneBody:
    radius: float
    n_src: int
    n_col: int
    r_src: float           # ring radius as a fraction of the disk radius
    Yr: np.ndarray         # (N_c, 2) sources relative to the centre
    Xr: np.ndarray         # (M_c, 2) nodes relative to the centre
    P: np.ndarray          # (2M_c, 2N_c) self block S(X, Y)
    K: np.ndarray          # (2N_c, 3)
    B: np.ndarray          # (2M_c, 3)
    IL: np.ndarray         # (2N_c, 2N_c) I - L
    U: np.ndarray
    s: np.ndarray
    Vt: np.ndarray
    problem: str

    def pinv(self, mu):
        """lambda_bar = P^+ mu (resistance) or S_L^+ mu (mobility), stably."""
        return apply_pinv(self.U, self.s, self.Vt, mu)

    def project(self, lam):
        """sigma = (I - L) lambda for mobility; identity for resistance (Sec. 4.4)."""
        if self.problem == "mobility":
            return self.IL @ lam
        return lam


def one_body(radius, n_src, n_col, r_src, mu, problem, eps_trunc, eps_ring=1e-12):
    """Build the shared one-body data of a radius class.  r_src <= 0 selects the ring rule of Sec. 6."""
    if r_src <= 0:
        r_src = ring_radius(n_src, eps_ring)
    Yr = ring((0.0, 0.0), r_src * radius, n_src)
    Xr = ring((0.0, 0.0), radius, n_col)
    P = stokeslet_matrix(Xr, Yr, mu)
    K = rigid_map(Yr, (0.0, 0.0))
    B = rigid_map(Xr, (0.0, 0.0))
    IL = np.eye(2 * n_src) - rigid_projector(K)
    if problem == "mobility":
        M = P @ IL + B @ K.T
    elif problem == "resistance":
        M = P
    else:
        raise ValueError(problem)
    U, s, Vt = truncated_svd(M, eps_trunc)
    return OneBody(radius, n_src, n_col, r_src, Yr, Xr, P, K, B, IL, U, s, Vt, problem)
