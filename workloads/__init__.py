"""Seeded synthetic planning problems shared by the HIP planner and the oracle.

This package only generates inputs (scene geometry, start/goal, bounds and
planner sizes).  It holds none of the planner's arithmetic: no dynamics, no
integration, no validity test, no sampling of controls.
"""

from .scenes import (  # noqa: F401
    batch_workloads,
    diff_workload,
    DiffBatch,
    DYNAMICS,
    COSTS,
    STATE_DIM,
    CONTROL_DIM,
    Problem,
    Params,
    Workload,
    di6_workload,
    quad12_workload,
    dubins6_workload,
    make_workload,
    WORKLOADS,
)
