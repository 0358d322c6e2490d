"""Per-pair precompute of the two-body correction (oracle).

For a near-contact pair (i, k) with coarse one-body data of each disk (unit disks as
in the paper; radius 1.4 disks by the reading taken for unequal radii), following Sec. 3.2-3.4 (resistance)
and Sec. 4.3-4.4 (mobility):

* X = [[0, Q^(k,i)], [Q^(i,k), 0]]: rows are the fine nodes of body i then body k,
  columns are lambda_bar^(i) then lambda_bar^(k) (Remark "Symmetrizing pairs").
  Resistance: Q^(i,k) = S(fine nodes of k, Y^(i)).  Mobility: Q^(i,k) =
  S(fine nodes of k, Y^(i)) (I - L) (eq. after Sec. 4.4 bullet list).
* F = S(fine nodes, fine sources) (resistance), or, for mobility,
  S(fine nodes, fine sources)(I - calL) + blockdiag(calB_i calK_i^T, calB_k calK_k^T)
  with calL the blockwise rigid projector of the fine sources (eq. chi_mob) and
  calB the fine-node rigid map (a reading: the text defines the fine counterpart).
* C = S(peanut, Y^(i) u Y^(k)) [(I - L^pair)],  D = S(peanut, fine sources) [(I - calL)]
  (eq. peanut / eq. peanut_mob).
* G = F^+ X with truncation 1e-11 (a reading of the paper), applied as V Sigma^+ (U^T X).
* A = -C^+ D G with truncation 1e-14 (eq. Amat), right to left (a reading of the paper).
* E: force/torque extraction (resistance) E_ft = -blockdiag(calK_i^T, calK_k^T) G,
  since beta = -F^+ X lambda_bar and f = K^T lambda_bar + calK^T beta (eq. force_syst);
  velocity extraction (mobility) E_v = +blockdiag(calK^T) G, since
  [v; omega] = -calK^T beta - K^T lambda_bar (eq. rbm2).  (A reading: eq. force_ext
  as printed lacks the transpose and the sign.)
* W: the step-2b field correction of Alg. 3 for this pair, precombined,
  W = -([[P, S^(ik)], [S^(ki), P]] Pi A + [[0, S^(ik) Pi], [S^(ki) Pi, 0]]) with
  Pi = I - L for mobility (a reading of the paper) and Pi = I for resistance, and with the
  H blocks of step 2b read as the one-body basis of the neighbour evaluated at
  the coarse nodes (a reading of the paper): H^(k,i) mu^(k) = S^(ik) Pi lambda_bar^(k).
"""

from __future__ import annotations

import numpy as np
from scipy.linalg import block_diag

from .geometry import fine_nodes, fine_sources, peanut_nodes, rigid_map, rigid_projector
from .kernel import stokeslet_matrix
from .onebody import apply_pinv, truncated_svd


def pair_matrices(ci, ck, ob, prm, keep=False, ob_k=None):
    """Precompute A, E and W for the pair (i, k): A (2N_i + 2N_k square), E (6 x (2N_i + 2N_k)),
    W ((2M_i + 2M_k) x (2N_i + 2N_k)).  ob is disk i's one-body data, ob_k disk k's (default: the
    same class).  Unequal radii follow the reading taken for unequal radii (limit points, fine counts scaled with the
    radius, a rolling unit circle for the peanut)."""
    ob_i = ob
    ob_k = ob if ob_k is None else ob_k
    ai, ak = float(ob_i.radius), float(ob_k.radius)
    ci = np.asarray(ci, dtype=np.float64)
    ck = np.asarray(ck, dtype=np.float64)
    mu = prm.mu
    mob = ob_i.problem == "mobility"
    Yi = ci + ob_i.Yr
    Yk = ck + ob_k.Yr
    Xi = ci + ob_i.Xr
    Xk = ck + ob_k.Xr
    Yfi, Yfk = fine_sources(ci, ck, prm, ai, ak)
    Xfi, Xfk = fine_nodes(ci, ck, prm, ai, ak)
    z = peanut_nodes(ci, ck, prm.m_p, ai, ak, rho=1.0)
    Yf = np.concatenate([Yfi, Yfk])
    Xf = np.concatenate([Xfi, Xfk])
    Kfi = rigid_map(Yfi, ci)
    Kfk = rigid_map(Yfk, ck)
    nci, nck = 2 * ob_i.n_src, 2 * ob_k.n_src
    Pi_i = ob_i.IL if mob else np.eye(nci)
    Pi_k = ob_k.IL if mob else np.eye(nck)

    Q_ik = stokeslet_matrix(Xfk, Yi, mu) @ Pi_i      # body i's basis on body k's fine nodes
    Q_ki = stokeslet_matrix(Xfi, Yk, mu) @ Pi_k      # body k's basis on body i's fine nodes
    mfi, mfk = 2 * Xfi.shape[0], 2 * Xfk.shape[0]
    Xmat = np.zeros((mfi + mfk, nci + nck))
    Xmat[:mfi, nci:] = Q_ki
    Xmat[mfi:, :nci] = Q_ik

    Sff = stokeslet_matrix(Xf, Yf, mu)
    Szf = stokeslet_matrix(z, Yf, mu)
    Szc = stokeslet_matrix(z, np.concatenate([Yi, Yk]), mu)
    if mob:
        ILf = block_diag(np.eye(Kfi.shape[0]) - rigid_projector(Kfi), np.eye(Kfk.shape[0]) - rigid_projector(Kfk))
        Bfi = rigid_map(Xfi, ci)
        Bfk = rigid_map(Xfk, ck)
        F = Sff @ ILf + block_diag(Bfi @ Kfi.T, Bfk @ Kfk.T)
        C = Szc @ block_diag(Pi_i, Pi_k)
        D = Szf @ ILf
    else:
        F = Sff
        C = Szc
        D = Szf

    UF, sF, VtF = truncated_svd(F, prm.eps_trunc_fine)
    G = apply_pinv(UF, sF, VtF, Xmat)
    UC, sC, VtC = truncated_svd(C, prm.eps_trunc)
    A = -apply_pinv(UC, sC, VtC, D @ G)
    KfT = block_diag(Kfi.T, Kfk.T)
    E = KfT @ G if mob else -(KfT @ G)

    Sik = stokeslet_matrix(Xi, Yk, mu)
    Ski = stokeslet_matrix(Xk, Yi, mu)
    near = np.block([[ob_i.P @ Pi_i, Sik @ Pi_k], [Ski @ Pi_i, ob_k.P @ Pi_k]])
    cross = np.block([[np.zeros((ob_i.P.shape[0], nci)), Sik @ Pi_k], [Ski @ Pi_i, np.zeros((ob_k.P.shape[0], nck))]])
    W = -(near @ A + cross)

    out = dict(A=A, E=E, W=W, n_fine=(Yfi.shape[0], Yfk.shape[0]))
    if keep:
        out.update(F=F, C=C, D=D, X=Xmat, G=G, sF=sF, sC=sC, Yf=Yf, Xf=Xf, z=z, Kfi=Kfi, Kfk=Kfk,
                   Yfi=Yfi, Yfk=Yfk, Xfi=Xfi, Xfk=Xfk)
    return out
