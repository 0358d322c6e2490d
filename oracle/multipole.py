"""Far field of one disk's ring of Stokeslets from its multipole moments (oracle).

Test infrastructure: a plain FP64 reference for the far-field expansion the library's
mixed kernel sum uses; only tests, the smoke check and the benchmark's CPU baseline use it.

The paper evaluates the all-pairs sum with a fast multipole method (Sec. 6); the library
evaluates the field of a far disk from the disk's own multipole moments (one level, no
tree).  In complex notation (x -> x_1 + i x_2, sigma = sigma_1 + i sigma_2) the Stokeslet of
eq. stokeslet2d applied to sigma at distance d = x - y is

  4 pi mu S(d) sigma = -sigma log|d| + sigma / 2 + conj(sigma) d / (2 conj(d)),

since (d . sigma) d / |d|^2 = (conj(sigma) d / conj(d) + sigma) / 2.  For sources
y_s = c + w_s on a ring |w_s| = rho and a point x = c + Z with |Z| > rho, put zeta = 1/Z,
A_k = sum_s sigma_s w_s^k (A_0 = S0, the net strength) and B_k = sum_s sigma_s conj(w_s)^k.
Then

  sum_s 4 pi mu S(x - y_s) sigma_s
    = -S0 log|Z| + S0/2 + sum_{k>=1} (A_k zeta^k + B_k conj(zeta)^k) / (2k)
      + conj(zeta)/2 [ (Z - rho^2 conj(zeta)) P - conj(B_1) ],
  P = sum_{k>=0} conj(A_k) conj(zeta)^k,

from log|1 - q| = -Re sum_k q^k / k, 1/(conj(Z) - conj(w)) = conj(zeta) sum_k (conj(w zeta))^k
and, on the ring, w = rho^2 / conj(w), which turns sum conj(sigma) w / (conj(Z) - conj(w)) into
conj(zeta) conj(B_1) + rho^2 conj(zeta)^2 P.  Truncating every series after k = p leaves an
error below about sum_s |sigma_s| theta^(p+1) / (1 - theta) (units of 4 pi mu), theta = rho/|Z|.
"""

from __future__ import annotations

import numpy as np


def moments(w, sigma, p):
    """A_0..A_p and B_0..B_p of complex offsets w (n,) and complex strengths sigma (n,)."""
    w = np.asarray(w, dtype=np.complex128)
    sigma = np.asarray(sigma, dtype=np.complex128)
    k = np.arange(p + 1)
    A = (sigma[None, :] * w[None, :] ** k[:, None]).sum(axis=1)
    B = (sigma[None, :] * np.conj(w)[None, :] ** k[:, None]).sum(axis=1)
    return A, B


def far_field(Z, A, B, rho, mu=1.0):
    """Velocity (complex, shape of Z) at offsets Z from the ring's centre, from moments A, B
    (length p + 1), truncated after order p."""
    Z = np.asarray(Z, dtype=np.complex128)
    p = len(A) - 1
    zeta = 1.0 / Z
    zb = np.conj(zeta)
    u = -A[0] * np.log(np.abs(Z)) + A[0] / 2
    for k in range(1, p + 1):
        u = u + (A[k] * zeta ** k + B[k] * zb ** k) / (2 * k)
    P = sum(np.conj(A[k]) * zb ** k for k in range(p + 1))
    u = u + zb / 2 * ((Z - rho * rho * zb) * P - np.conj(B[1]))
    return u / (4 * np.pi * mu)


def cluster_moments(w, sigma, p):
    """Moments of sources at arbitrary offsets w (n,) from an expansion centre (a cluster of
    disks): A_k = sum sigma w^k, B_k = sum sigma conj(w)^k and D_k = sum sigma conj(w) w^k,
    k = 0..p."""
    w = np.asarray(w, dtype=np.complex128)
    sigma = np.asarray(sigma, dtype=np.complex128)
    A, B = moments(w, sigma, p)
    k = np.arange(p + 1)
    D = (sigma[None, :] * np.conj(w)[None, :] * w[None, :] ** k[:, None]).sum(axis=1)
    return A, B, D


def far_field_general(Z, A, B, D, mu=1.0):
    """Velocity (complex) at offsets Z from the centre of sources that need not lie on a ring,
    from cluster_moments, truncated after order p = len(A) - 1.

    The third term of the Stokeslet sums conj(sigma) (Z - w) / (conj(Z) - conj(w)); with
    1/(conj(Z) - conj(w)) = conj(zeta) sum_k (conj(w zeta))^k it is
    conj(zeta) [Z sum_k conj(A_k) conj(zeta)^k - sum_k conj(D_k) conj(zeta)^k], so

      4 pi mu u = -S0 log|Z| + S0/2 + sum_{k>=1} (A_k zeta^k + B_k conj(zeta)^k) / (2k)
                  + conj(zeta)/2 [Z P - Q],  P = sum conj(A_k) conj(zeta)^k,
                                             Q = sum conj(D_k) conj(zeta)^k.

    On a ring |w| = rho, D_k = rho^2 A_{k-1} (k >= 1) and D_0 = B_1, which gives far_field.
    Truncation: below about sum |sigma| theta^(p+1) / (1 - theta), theta = max|w| / |Z|."""
    Z = np.asarray(Z, dtype=np.complex128)
    p = len(A) - 1
    zeta = 1.0 / Z
    zb = np.conj(zeta)
    u = -A[0] * np.log(np.abs(Z)) + A[0] / 2
    for k in range(1, p + 1):
        u = u + (A[k] * zeta ** k + B[k] * zb ** k) / (2 * k)
    P = sum(np.conj(A[k]) * zb ** k for k in range(p + 1))
    Q = sum(np.conj(D[k]) * zb ** k for k in range(p + 1))
    u = u + zb / 2 * (Z * P - Q)
    return u / (4 * np.pi * mu)
