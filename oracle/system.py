"""The global preconditioned system, its matvec, RHS, post-processing and GMRES (oracle).

The unknown is mu = {mu^(i)}: coarse collocation data, 2 M_c values per body,
per node (x, y) interleaved, body-major (a reading of the paper).

``matvec`` is Alg. 3 step by step (with the mobility projections of Sec. 4.4):
 1a  lambda_bar^(i) = P^+ mu^(i)  (mobility: S_L^+ mu^(i)),  lambda = lambda_bar
 1b  for each close pair c = (i, k): lambda_tilde^c = A^c [lambda_bar^(i); lambda_bar^(k)],
     added to lambda^(i), lambda^(k)                        (eq. correction, eq. total_corr)
 2a  u = sum over all bodies of S(X, Y^(k)) Pi lambda^(k), self included (eq. getall)
 2b  for each pair: u_pair -= [[P, S^(ik)], [S^(ki), P]] Pi lambda_tilde^c
                              + [[0, H^(k,i)], [H^(i,k), 0]] [mu^(i); mu^(k)]
     identity fix: u^(i) += mu^(i) - P Pi lambda_bar^(i)     (eq. onesub)
where Pi = I - L for mobility (a reading of the paper) and Pi = I for resistance, and
H^(k,i) mu^(k) = S^(ik) Pi lambda_bar^(k) (a reading of the paper).

``matvec_masked`` is the closed form these steps collapse to in exact arithmetic:
  (T mu)^(i) = mu^(i) + sum_{k not i, k not a neighbour of i} S^(ik) Pi lambda_bar^(k)
                     + sum_{pairs c not containing i} sum_{k in c} S^(ik) Pi lambda_tilde^c_k,
an independent assembly used to pin the bookkeeping of step 2b.

RHS (mobility, Sec. 4.1-4.2): lambda_0^(i) = K (K^T K)^{-1} [f; t]^(i) (so that
K^T lambda_0 = [f; t]), u_0 = S lambda_0 summed over all bodies with self
(eq. u0_def), b = -u_0 (a reading of the paper).  Resistance: b^(i) = B [v; omega]^(i)
(eq. rigidbc at the coarse nodes).

Post-processing: mobility [v; omega]^(i) = -K^T lambda_bar^(i) + sum_{c contains i}
(E_v^c x_c)_i (eq. rbm_ansatz, eq. rbm2, a reading of the paper); resistance
[f; t]^(i) = K^T lambda_bar^(i) + sum_c (E_ft^c x_c)_i (eq. two_force, Alg. 2).
Forces are the sums of Stokeslet strengths, i.e. the force exerted on the fluid
(a reading of the paper).
"""

from __future__ import annotations

import math
import time

import numpy as np

from .geometry import contacts
from .kernel import direct_sum, stokeslet_matrix
from .onebody import one_body
from .pairs import pair_matrices
from .params import MFSParams


class System:
    """Geometry, one-body classes, contacts and pair matrices of one suspension."""

    def __init__(self, centers, radii, n_src, n_col, r_src, problem, prm=MFSParams(),
                 pair_data=None, progress=False):
        self.c = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 2)
        P = self.c.shape[0]
        self.P = P
        self.a = np.broadcast_to(np.asarray(radii, dtype=np.float64), (P,)).copy()
        self.n_src = np.broadcast_to(np.asarray(n_src, dtype=np.int64), (P,)).copy()
        self.n_col = np.broadcast_to(np.asarray(n_col, dtype=np.int64), (P,)).copy()
        self.r_src = np.broadcast_to(np.asarray(r_src, dtype=np.float64), (P,)).copy()
        self.problem = problem
        self.prm = prm
        keys = [(float(self.a[i]), int(self.n_src[i]), int(self.n_col[i]), float(self.r_src[i])) for i in range(P)]
        self.classes = {}
        self.cls = []
        for key in keys:
            if key not in self.classes:
                self.classes[key] = one_body(key[0], key[1], key[2], key[3], prm.mu, problem, prm.eps_trunc,
                                             prm.eps_ring)
            self.cls.append(self.classes[key])
        self.src_off = np.concatenate([[0], np.cumsum(self.n_src)])
        self.col_off = np.concatenate([[0], np.cumsum(self.n_col)])
        self.Y = np.concatenate([self.c[i] + self.cls[i].Yr for i in range(P)])
        self.X = np.concatenate([self.c[i] + self.cls[i].Xr for i in range(P)])
        self.n = 2 * int(self.col_off[-1])
        self.pairs = contacts(self.c, self.a, prm.delta_c)
        self.neigh = [set() for _ in range(P)]
        for i, k in self.pairs:
            self.neigh[i].add(int(k))
            self.neigh[k].add(int(i))
        t0 = time.time()
        if pair_data is None:
            pair_data = []
            for idx, (i, k) in enumerate(self.pairs):
                pair_data.append(pair_matrices(self.c[i], self.c[k], self.cls[i], prm, ob_k=self.cls[k]))
                if progress and idx % 50 == 0:
                    print(f"  pair {idx}/{len(self.pairs)}  {time.time() - t0:.1f}s", flush=True)
        self.pd = pair_data
        self.t_precompute = time.time() - t0

    # -- slicing helpers ---------------------------------------------------------
    def mu_of(self, v, i):
        return v[2 * self.col_off[i]:2 * self.col_off[i + 1]]

    def src_of(self, v, i):
        return v[2 * self.src_off[i]:2 * self.src_off[i + 1]]

    def Yb(self, i):
        return self.Y[self.src_off[i]:self.src_off[i + 1]]

    def Xb(self, i):
        return self.X[self.col_off[i]:self.col_off[i + 1]]

    # -- Alg. 3 ------------------------------------------------------------------
    def step1(self, mu):
        """Steps 1a and 1b: lambda_bar, lambda and the per-pair lambda_tilde."""
        lam_bar = np.concatenate([self.cls[i].pinv(self.mu_of(mu, i)) for i in range(self.P)])
        lam = lam_bar.copy()
        ltil = []
        for c, (i, k) in enumerate(self.pairs):
            x = np.concatenate([self.src_of(lam_bar, i), self.src_of(lam_bar, k)])
            t = self.pd[c]["A"] @ x
            ni = 2 * self.n_src[i]
            self.src_of(lam, i)[:] += t[:ni]
            self.src_of(lam, k)[:] += t[ni:]
            ltil.append(t)
        return lam_bar, lam, ltil

    def sigma(self, lam):
        return np.concatenate([self.cls[i].project(self.src_of(lam, i)) for i in range(self.P)])

    def matvec(self, mu, workers=None):
        """T mu by Alg. 3 (FP64, direct O(N_s N_t) sum in step 2a)."""
        mu = np.asarray(mu, dtype=np.float64)
        lam_bar, lam, ltil = self.step1(mu)
        sig = self.sigma(lam).reshape(-1, 2)
        # sources of zero strength add nothing to eq. getall: leaving them out changes no
        # term of the sum (it lets inputs supported on a few disks run at large P)
        nz = np.any(sig != 0.0, axis=1)
        u = direct_sum(self.X, self.Y[nz], sig[nz], self.prm.mu, workers=workers).reshape(-1)
        mu_v = self.prm.mu
        for c, (i, k) in enumerate(self.pairs):
            ni = 2 * self.n_src[i]
            ti, tk = ltil[c][:ni], ltil[c][ni:]
            obi, obk = self.cls[i], self.cls[k]
            Sik = stokeslet_matrix(self.Xb(i), self.Yb(k), mu_v)
            Ski = stokeslet_matrix(self.Xb(k), self.Yb(i), mu_v)
            self.mu_of(u, i)[:] -= obi.P @ obi.project(ti) + Sik @ obk.project(tk) \
                + Sik @ obk.project(self.src_of(lam_bar, k))
            self.mu_of(u, k)[:] -= Ski @ obi.project(ti) + obk.P @ obk.project(tk) \
                + Ski @ obi.project(self.src_of(lam_bar, i))
        for i in range(self.P):
            ob = self.cls[i]
            self.mu_of(u, i)[:] += self.mu_of(mu, i) - ob.P @ ob.project(self.src_of(lam_bar, i))
        return u

    def matvec_masked(self, mu):
        """Closed masked form of T mu (dense block loops; small P only)."""
        mu = np.asarray(mu, dtype=np.float64)
        lam_bar, _, ltil = self.step1(mu)
        u = mu.copy()
        mu_v = self.prm.mu
        for i in range(self.P):
            acc = np.zeros(2 * self.n_col[i])
            for k in range(self.P):
                if k == i or k in self.neigh[i]:
                    continue
                acc += stokeslet_matrix(self.Xb(i), self.Yb(k), mu_v) @ self.cls[k].project(self.src_of(lam_bar, k))
            for c, (p, q) in enumerate(self.pairs):
                if i in (p, q):
                    continue
                npq = 2 * self.n_src[p]
                for k, part in ((p, ltil[c][:npq]), (q, ltil[c][npq:])):
                    acc += stokeslet_matrix(self.Xb(i), self.Yb(k), mu_v) @ self.cls[k].project(part)
            self.mu_of(u, i)[:] += acc
        return u

    def matvec_W(self, mu, workers=None):
        """Alg. 3 with the step-2b loop applied through the precombined W^c."""
        mu = np.asarray(mu, dtype=np.float64)
        lam_bar, lam, _ = self.step1(mu)
        sig = self.sigma(lam)
        u = direct_sum(self.X, self.Y, sig.reshape(-1, 2), self.prm.mu, workers=workers).reshape(-1)
        for c, (i, k) in enumerate(self.pairs):
            x = np.concatenate([self.src_of(lam_bar, i), self.src_of(lam_bar, k)])
            w = self.pd[c]["W"] @ x
            mi = 2 * self.n_col[i]
            self.mu_of(u, i)[:] += w[:mi]
            self.mu_of(u, k)[:] += w[mi:]
        for i in range(self.P):
            ob = self.cls[i]
            self.mu_of(u, i)[:] += self.mu_of(mu, i) - ob.P @ ob.project(self.src_of(lam_bar, i))
        return u

    def dense(self, masked=False):
        """Assemble T column by column (small P only)."""
        T = np.empty((self.n, self.n))
        e = np.zeros(self.n)
        f = self.matvec_masked if masked else (lambda v: self.matvec(v, workers=1))
        for j in range(self.n):
            e[j] = 1.0
            T[:, j] = f(e)
            e[j] = 0.0
        return T

    # -- right-hand side and post-processing ----------------------------------------
    def rhs(self, given, workers=None):
        """Right-hand side b from (P, 3) forces/torques (mobility) or velocities (resistance)."""
        given = np.asarray(given, dtype=np.float64).reshape(self.P, 3)
        if self.problem == "mobility":
            lam0 = np.concatenate([ob.K @ np.linalg.solve(ob.K.T @ ob.K, given[i]) for i, ob in enumerate(self.cls)])
            u0 = direct_sum(self.X, self.Y, lam0.reshape(-1, 2), self.prm.mu, workers=workers).reshape(-1)
            return -u0
        return np.concatenate([ob.B @ given[i] for i, ob in enumerate(self.cls)])

    def post(self, mu):
        """(P, 3) velocities (mobility) or forces/torques (resistance) from the solution mu."""
        lam_bar = np.concatenate([self.cls[i].pinv(self.mu_of(mu, i)) for i in range(self.P)])
        sgn = -1.0 if self.problem == "mobility" else 1.0
        out = np.stack([sgn * (self.cls[i].K.T @ self.src_of(lam_bar, i)) for i in range(self.P)])
        for c, (i, k) in enumerate(self.pairs):
            x = np.concatenate([self.src_of(lam_bar, i), self.src_of(lam_bar, k)])
            e = self.pd[c]["E"] @ x
            out[i] += e[:3]
            out[k] += e[3:]
        return out


def gmres(matvec, b, tol, maxit=500, x0=None, callback=None):
    """Unrestarted GMRES (modified Gram-Schmidt Arnoldi, Givens rotations; the paper does not fix the variant).

    Stops when the Givens residual estimate |g_{k+1}| <= tol * |b|.  Returns
    (x, info) with info = dict(iters, resid (estimates), true_resid).
    """
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    r = b - matvec(x) if x0 is not None else b.copy()
    beta = np.linalg.norm(r)
    bnorm = np.linalg.norm(b)
    hist = [beta / bnorm if bnorm > 0 else 0.0]
    if bnorm == 0.0:
        return np.zeros(n), dict(iters=0, resid=hist, true_resid=0.0)
    m = maxit
    V = np.zeros((m + 1, n))
    H = np.zeros((m + 1, m))
    cs = np.zeros(m)
    sn = np.zeros(m)
    g = np.zeros(m + 1)
    g[0] = beta
    V[0] = r / beta
    k_done = 0
    for k in range(m):
        w = matvec(V[k])
        for j in range(k + 1):
            H[j, k] = V[j] @ w
            w = w - H[j, k] * V[j]
        H[k + 1, k] = np.linalg.norm(w)
        if H[k + 1, k] > 0:
            V[k + 1] = w / H[k + 1, k]
        for j in range(k):
            t = cs[j] * H[j, k] + sn[j] * H[j + 1, k]
            H[j + 1, k] = -sn[j] * H[j, k] + cs[j] * H[j + 1, k]
            H[j, k] = t
        den = math.hypot(H[k, k], H[k + 1, k])
        cs[k] = H[k, k] / den
        sn[k] = H[k + 1, k] / den
        H[k, k] = den
        H[k + 1, k] = 0.0
        g[k + 1] = -sn[k] * g[k]
        g[k] = cs[k] * g[k]
        k_done = k + 1
        hist.append(abs(g[k + 1]) / bnorm)
        if callback is not None:
            callback(k_done, hist[-1])
        if abs(g[k + 1]) <= tol * bnorm or H[k, k] == 0.0:
            break
    y = np.zeros(k_done)
    for j in range(k_done - 1, -1, -1):
        y[j] = (g[j] - H[j, j + 1:k_done] @ y[j + 1:]) / H[j, j]
    x = x + V[:k_done].T @ y
    true_resid = np.linalg.norm(b - matvec(x)) / bnorm
    return x, dict(iters=k_done, resid=hist, true_resid=true_resid)


def rel_rigid_error(out, ref):
    """eq. rel_vel_err: E^(i) = (|v - v_ref| + |omega - omega_ref|) / max_j s_ref^(j), s = |v| + |omega|."""
    out = np.asarray(out, dtype=np.float64).reshape(-1, 3)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1, 3)
    e = np.linalg.norm(out[:, :2] - ref[:, :2], axis=1) + np.abs(out[:, 2] - ref[:, 2])
    s = np.linalg.norm(ref[:, :2], axis=1) + np.abs(ref[:, 2])
    return e / s.max()


def solve(system, given, tol, maxit=500, workers=None, callback=None):
    """Alg. 2 / Sec. 4.4 solve: RHS, GMRES on Alg. 3, post-processing.  Returns (out (P,3), mu, info)."""
    b = system.rhs(given, workers=workers)
    mu, info = gmres(lambda v: system.matvec(v, workers=workers), b, tol, maxit, callback=callback)
    return system.post(mu), mu, info
