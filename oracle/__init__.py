"""FP64 CPU oracle of the peanut-compressed two-body MFS (test infrastructure only).

This package is a plain, slow, obviously-correct NumPy/SciPy implementation of
what the MI355X path computes.  It exists to check that path.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The product library never calls it and shares no code with it.  The
two sides are independent implementations of the same readings of the paper.
The only inputs they share come from the ``workloads`` package: centres, radii
and right-hand sides.

Layout, each module citing the passages it follows:

* ``kernel``    -- 2D Stokeslet (eq. stokeslet2d) and plain direct sums (eq. stokes_sum).
* ``geometry``  -- coarse rings, rigid-body maps (eq. Kmat), contacts, fine sources
  and nodes (Sec. 5), peanut nodes (Sec. 3.3).
* ``onebody``   -- one-body bases: P^+ (Sec. 3.1, eq. howG+) and S_L^+ (Sec. 4.1, eq. SL).
* ``pairs``     -- per-pair precompute: F, Q, C, D and the compressed A (eq. Amat),
  E (eq. force_ext / eq. rbm2), and the step-2b field-correction matrix W.
* ``system``    -- Alg. 3 matvec, its closed masked form, RHS, post-processing,
  GMRES and the error metric of eq. rel_vel_err.
* ``direct``    -- brute-force fine-grid MFS solves used only as pins.

Readings of passages that are silent, ambiguous or garbled are listed in each
docstring where they apply.  Every function here has at least one pin in
``tests/test_oracle_*.py``.
"""

from .kernel import stokeslet_blocks, stokeslet_matrix, direct_sum  # noqa: F401
from .params import MFSParams  # noqa: F401
