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

import math

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


def local_expansion(A, B, D, Delta, q):
    """Local (Taylor) expansion about a point T of the field of sources with cluster_moments
    A, B, D about C, Delta = T - C (complex, |Delta| > the sources' radius), to order q.

    far_field_general is, with Z = x - C and F(Z) = sum_{k>=0} A_k Z^-(k+1),
      4 pi mu u = Phi1(Z) + conj(Phi2(Z)) - Z conj(Phi1'(Z)) + A_0 / 2,
      Phi1 = -(A_0/2) log Z + sum_{k>=1} A_k Z^-k / (2k),           Phi1' = -F / 2,
      Phi2 = -(conj(A_0)/2) log Z + sum_{k>=1} conj(B_k) Z^-k / (2k) - (1/2) sum_{k>=0} D_k Z^-(k+1),
    (Goursat's form of a plane Stokes flow).  Writing Z = w + Delta with w = x - T moves the
    non-analytic factor to the target side: -Z conj(Phi1') = -w conj(Phi1') + conj(-conj(Delta) Phi1'),
    so with Psi = Phi2 - conj(Delta) Phi1' (analytic near T)
      4 pi mu u = Phi1 + conj(Psi) - w conj(Phi1') + A_0 / 2.
    Each of f = Phi1, Psi is a log term a log Z plus sum_k c_k Z^-k; about T
      log(w + Delta) = log Delta - sum_{l>=1} (-w/Delta)^l / l,
      (w + Delta)^-k = sum_{l>=0} (-1)^l binom(k + l - 1, l) Delta^-(k+l) w^l.
    Only Re log enters u (the imaginary parts of Phi1's and conj(Psi)'s log terms cancel), so
    log Delta is taken as log|Delta|.  Returns (L1, L2, const): the coefficients of w^0..w^q of
    Phi1 and Psi and A_0 / 2."""
    A = np.asarray(A, dtype=np.complex128)
    B = np.asarray(B, dtype=np.complex128)
    D = np.asarray(D, dtype=np.complex128)
    p = len(A) - 1
    Delta = complex(Delta)
    a1 = -A[0] / 2
    a2 = -np.conj(A[0]) / 2
    c1 = np.zeros(p + 2, dtype=np.complex128)
    c2 = np.zeros(p + 2, dtype=np.complex128)
    for k in range(1, p + 2):
        if k <= p:
            c1[k] = A[k] / (2 * k)
            c2[k] += np.conj(B[k]) / (2 * k)
        c2[k] += -D[k - 1] / 2 + np.conj(Delta) * A[k - 1] / 2

    def taylor(a, c):
        L = np.zeros(q + 1, dtype=np.complex128)
        L[0] = a * math.log(abs(Delta)) + sum(c[k] * Delta ** (-k) for k in range(1, p + 2))
        for l in range(1, q + 1):
            L[l] = -a * (-1) ** l / (l * Delta ** l) + sum(
                c[k] * (-1) ** l * math.comb(k + l - 1, l) * Delta ** (-k - l) for k in range(1, p + 2))
        return L

    return taylor(a1, c1), taylor(a2, c2), A[0] / 2


def eval_local(w, L1, L2, const, mu=1.0):
    """Velocity (complex) at offsets w from the expansion point of a local expansion
    (local_expansion, or a sum of several): u = L1(w) + conj(L2(w)) - w conj(L1'(w)) + const,
    in units of 1 / (4 pi mu)."""
    w = np.asarray(w, dtype=np.complex128)
    q = len(L1) - 1
    v1 = sum(L1[l] * w ** l for l in range(q + 1))
    d1 = sum(l * L1[l] * w ** (l - 1) for l in range(1, q + 1))
    v2 = sum(L2[l] * w ** l for l in range(q + 1))
    return (v1 + np.conj(v2) - w * np.conj(d1) + const) / (4 * np.pi * mu)
