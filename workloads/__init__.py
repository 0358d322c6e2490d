"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package generates geometry (disk centres and radii) and right-hand-side draws
only.  It holds none of the method's arithmetic: no Stokeslet, no discretisation
of the disks, no linear algebra of the solver.  Both the FP64 CPU oracle and the
HIP path consume what it returns, so that the two are compared on identical
inputs.
"""

from .packings import (  # noqa: F401
    jittered_grid,
    lattice_packing,
    bidisperse_packing,
    min_gap,
    close_pairs_count,
    config_geometry,
    CONFIG_SEED_BASE,
)
from .rhs import (  # noqa: F401
    mobility_rhs,
    resistance_rhs,
    unit_torques,
)
from .serving import (  # noqa: F401
    serving_request,
    poisson_arrivals,
    SERVING_SEED_BASE,
)
