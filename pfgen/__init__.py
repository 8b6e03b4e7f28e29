"""Seeded synthetic power-flow inputs.

This module makes the grids that both the GPU library and the CPU oracle are
run on. It holds no part of the Newton power-flow method itself: it draws
topologies, branch impedances, bus types and set-points from a seed and stamps
the nodal admittance matrix that the library takes as input (the nodal
equation and the admittance assembly of Sec. II, eq. 1-3 and eq. 11).

The paper's own cases (IEEE-30 replicas, Sec. IV; IEEE 906 LV feeder
replicas, Sec. IV) are not available, so seeded synthetic grids of the same
kind stand in for them. The recipe for every workload is in ``grids.py``.
"""

from .grids import (  # noqa: F401
    BASE_SEED,
    PolarCase,
    CimCase,
    make_polar_grid,
    make_feeder,
    config_case,
    perturb_loads,
    c3_scenarios,
    c4_pool,
    replicate_polar,
    add_dg_and_delta,
    replicate_feeder,
    replication_polar,
    replication_feeder,
    FEEDER_COPIES,
    replication_feeder_tol,
    PQ,
    PV,
    SLACK,
)
