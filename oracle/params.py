"""Method parameters with the paper's defaults (oracle copy).

Sec. 6 and Sec. 6.2: N_fp = 150, N_ell = 80, M_p = 200, SVD truncation 1e-14
(1e-11 for the fine solve), ring-radius rule with eps = 1e-12, contact threshold
0.2.  Sec. 5: gamma = 0.3, a_f = 1.2, Moebius parameter r = 0.6, a_ell = 5.
"""

from __future__ import annotations

from dataclasses import dataclass


@dataclass(frozen=True)
class MFSParams:
    mu: float = 1.0                 # dynamic viscosity
    delta_c: float = 0.2            # near-contact threshold on the gap
    eps_trunc: float = 1e-14        # one-body and peanut pseudoinverse truncation
    eps_trunc_fine: float = 1e-11   # fine pair pseudoinverse truncation
    eps_ring: float = 1e-12         # ring radius rule R = 1 - ln(1/eps)/N
    n_fp: int = 150                 # fine proxy sources per disk
    n_ell: int = 80                 # ellipse sampling parameter
    m_p: int = 200                  # peanut collocation nodes
    gamma: float = 0.3              # ellipse tip parameter
    a_f: float = 1.2                # equispaced fine nodes = ceil(a_f * n_fp)
    mobius_r: float = 0.6           # Moebius clustering parameter
    a_ell: int = 5                  # Moebius nodes = a_ell * n_ell
