"""Kino-PAX+ planner hot path on AMD Instinct MI355X.

The planner runs in libkpx.so (HIP kernels for gfx950 behind the C ABI in
include/kpx.h); this package only marshals arguments to it.
"""

from .kpx import (  # noqa: F401
    ACTIVE, INACTIVE, TERMINAL, Batch, KPXError, Planner, lib, philox, workspace_bytes,
    status_string, OK, FULL,
)
from .diff import Rollout, edge_loss  # noqa: F401,E402
