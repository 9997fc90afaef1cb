"""Kino-PAX+ planner hot path on AMD Instinct MI355X.

The planner runs in libkpx.so (HIP kernels for gfx950 behind the C ABI in
include/kpx.h); this package only marshals arguments to it.

One query (the problem and parameters are the dataclasses of workloads.scenes,
or any objects with the same fields):

    import paper_2602_02846_amd as kpx
    import workloads

    w = workloads.make_workload("quad12", 0)
    pl = kpx.Planner(w.problem, w.params)   # kpx_create on the current stream
    pl.iterate(200)                         # kpx_iterate: enqueued, returns at once
    sol = pl.solution()                     # kpx_solution: waits
    if sol["found"]:
        print(sol["cost"], sol["steps"], sol["controls"])
    pl.close()

Planner also offers snapshot / read_dump (tree and per-slot records),
set_timing / read_timing / stats (measurement), set_cost_first, set_polish and
refine; Batch iterates many planners together; Rollout and edge_loss give the
differentiable quadrotor edge rollout.
"""

from .kpx import (  # noqa: F401
    ACTIVE, INACTIVE, TERMINAL, Batch, KPXError, Planner, lib, philox, workspace_bytes,
    status_string, OK, FULL, ERR_ARG, PHILOX_STATIC_MAX, philox_static,
)
from .diff import Rollout, edge_loss  # noqa: F401,E402
