"""Seeded scene and planner-size generators for the three robot models.

Every constant is stored as a float32 value: the planner and the oracle both
read these exact values (the oracle widens them to float64), so no constant is
rounded differently on the two sides.

Scenes stand in for the paper's four environments (Sec. V, Forest / Narrow /
House / Zig-Zag), whose geometry is only shown in figures.  The generators
follow the shapes of the benchmark workloads:

* ``di6``     -- 6D double integrator, unit cube, 8 random boxes, 30^3 regions,
                 256 nodes x 8 samples per iteration, cost = time.
* ``quad12``  -- 12D quadrotor, unit cube with a wall of 64 boxes leaving two
                 0.08-wide slots, 16^3 x 2^3 regions, 4096 x 32 samples.
* ``dubins6`` -- 6D Dubins-airplane-like model, 200 building boxes,
                 32 x 32 x 16 regions, 8192 x 32 samples, cost = path length.

Random numbers for scene geometry come from numpy's PCG64 seeded with
``(seed, tag)``; they are independent of the planner's own control samples.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional

import numpy as np

DYNAMICS = {"DI6": 0, "QUAD12": 1, "DUBINS6": 2}
COSTS = {"TIME": 0, "PATH_LENGTH": 1}
STATE_DIM = {"DI6": 6, "QUAD12": 12, "DUBINS6": 6}
CONTROL_DIM = {"DI6": 3, "QUAD12": 4, "DUBINS6": 3}

MAX_STATE = 12
MAX_CONTROL = 4
INF = np.float32(np.inf)


def _f32(values, size: int, fill=0.0) -> np.ndarray:
    out = np.full(size, fill, dtype=np.float32)
    v = np.asarray(values, dtype=np.float32).ravel()
    out[: v.size] = v
    return out


@dataclasses.dataclass
class Problem:
    """Problem 1 of the paper: dynamics, valid set, start, goal set, cost."""

    dynamics: str
    cost: str
    dyn_params: np.ndarray  # float32[8]; QUAD12: m, Ixx, Iyy, Izz, g
    x_init: np.ndarray  # float32[12]
    x_lo: np.ndarray  # float32[12] (-inf allowed)
    x_hi: np.ndarray  # float32[12] (+inf allowed)
    u_lo: np.ndarray  # float32[4]
    u_hi: np.ndarray  # float32[4]
    ws_lo: np.ndarray  # float32[3]
    ws_hi: np.ndarray  # float32[3]
    boxes: np.ndarray  # float32[n, 6]: lo xyz, hi xyz
    margin: float  # planning clearance margin
    goal_center: np.ndarray  # float32[3]
    goal_radius: float

    @property
    def state_dim(self) -> int:
        return STATE_DIM[self.dynamics]

    @property
    def control_dim(self) -> int:
        return CONTROL_DIM[self.dynamics]

    @property
    def n_boxes(self) -> int:
        return int(self.boxes.shape[0])


@dataclasses.dataclass
class Params:
    """Algorithm parameters (Alg. 1 inputs plus the GPU sizing knobs)."""

    dt: float
    steps_min: int
    steps_max: int
    grid: tuple  # cells per position axis
    vel_sign_bins: int  # 1: 3 velocity-sign bits appended to the cell index
    n_select: int  # nodes expanded per iteration (at most)
    samples_per_node: int  # K
    tree_cap: int
    i_max: int
    seed: int
    query_id: int = 0
    refine_max: int = 0  # largest total grid refinement factor per axis (0/1: none)

    @property
    def n_cells(self) -> int:
        g = self.grid
        return int(g[0]) * int(g[1]) * int(g[2]) * (8 if self.vel_sign_bins else 1)

    @property
    def n_slots(self) -> int:
        """Candidate slots per iteration at most: n_select * K, or n_select
        (the buffer shared out among all active nodes) when K = 0."""
        return int(self.n_select) * max(1, int(self.samples_per_node))


@dataclasses.dataclass
class Workload:
    name: str
    problem: Problem
    params: Params
    iterations: int


def _rng(seed: int, tag: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed) & 0xFFFFFFFF, tag]))


def _box_hits_ball(box, c, r) -> bool:
    lo, hi = box[:3], box[3:]
    q = np.clip(c, lo, hi)
    return float(np.linalg.norm(q - c)) <= r


def _random_boxes(rng, n, center_lo, center_hi, side_lo, side_hi, start, goal_c, goal_r,
                  clear=0.02):
    boxes = []
    while len(boxes) < n:
        c = rng.uniform(center_lo, center_hi, size=3)
        s = rng.uniform(side_lo, side_hi, size=3)
        b = np.concatenate([c - s / 2, c + s / 2])
        if _box_hits_ball(b, start, clear) or _box_hits_ball(b, goal_c, goal_r + clear):
            continue
        boxes.append(b)
    return np.asarray(boxes, dtype=np.float32).reshape(n, 6)


def di6_workload(seed: int = 0, *, n_boxes: int = 8, n_select: int = 256, samples: int = 8,
                 tree_cap: int = 1 << 17, grid=(30, 30, 30), iterations: int = 200,
                 i_max: int = 10, cost: str = "TIME", margin: float = 1e-4,
                 steps=(5, 30)) -> Workload:
    """6D double integrator: p' = v, v' = u, u in [-1,1]^3, |v_i| <= 1.

    Regions: 30^3 over position (27,000 regions, the paper's large-delta
    setting for this system, App. B).  An 8^3 grid cannot be used: from rest,
    an edge of at most 0.3 s at |u| <= 1 moves at most 0.045, less than the
    0.075 to the start region's face, and every arrival inside the start region
    costs more than the region's best, so the tree would never grow."""
    start = np.array([0.05, 0.05, 0.05], dtype=np.float64)
    goal_c = np.array([0.95, 0.95, 0.95], dtype=np.float64)
    goal_r = 0.05
    rng = _rng(seed, 0xD16)
    boxes = _random_boxes(rng, n_boxes, 0.1, 0.9, 0.05, 0.15, start, goal_c, goal_r)
    prob = Problem(
        dynamics="DI6", cost=cost,
        dyn_params=_f32([], 8),
        x_init=_f32([0.05, 0.05, 0.05, 0, 0, 0], MAX_STATE),
        x_lo=_f32([-INF, -INF, -INF, -1, -1, -1], MAX_STATE),
        x_hi=_f32([INF, INF, INF, 1, 1, 1], MAX_STATE),
        u_lo=_f32([-1, -1, -1], MAX_CONTROL), u_hi=_f32([1, 1, 1], MAX_CONTROL),
        ws_lo=_f32([0, 0, 0], 3), ws_hi=_f32([1, 1, 1], 3),
        boxes=boxes, margin=float(np.float32(margin)),
        goal_center=_f32(goal_c, 3), goal_radius=float(np.float32(goal_r)),
    )
    prm = Params(dt=float(np.float32(0.01)), steps_min=steps[0], steps_max=steps[1],
                 grid=tuple(grid), vel_sign_bins=0, n_select=n_select,
                 samples_per_node=samples, tree_cap=tree_cap, i_max=i_max, seed=seed)
    return Workload("di6", prob, prm, iterations)


def _wall_boxes(rng, layers: int = 8, per_layer: int = 8, x0=0.48, x1=0.52, slot=0.08):
    while True:
        y1, y2 = np.sort(rng.uniform(0.15, 0.85, size=2))
        if y2 - y1 >= 0.2:
            break
    h = slot / 2
    segs = [(0.0, y1 - h), (y1 + h, y2 - h), (y2 + h, 1.0)]
    lens = np.array([b - a for a, b in segs])
    # every segment gets at least one box; the rest by largest remainder
    counts = np.ones(3, dtype=int)
    extra = per_layer - 3
    share = lens / lens.sum() * extra
    counts += np.floor(share).astype(int)
    rem = per_layer - counts.sum()
    for i in np.argsort(-(share - np.floor(share)))[:rem]:
        counts[i] += 1
    boxes = []
    for layer in range(layers):
        z0, z1 = layer / layers, (layer + 1) / layers
        for (a, b), c in zip(segs, counts):
            edges = np.linspace(a, b, c + 1)
            for k in range(c):
                boxes.append([x0, edges[k], z0, x1, edges[k + 1], z1])
    return np.asarray(boxes, dtype=np.float32), (float(y1), float(y2))


def quad12_workload(seed: int = 0, *, n_select: int = 4096, samples: int = 32,
                    tree_cap: int = 1 << 21, grid=(16, 16, 16), vel_sign_bins: int = 1,
                    iterations: int = 200, i_max: int = 10, margin: float = 1e-4,
                    steps=(5, 60), cost: str = "TIME") -> Workload:
    """12D quadrotor (ZYX Euler angles, world-frame velocity, body rates)."""
    m, inertia, g = 1.0, 0.01, 9.81
    rng = _rng(seed, 0x412)
    boxes, _ = _wall_boxes(rng)
    prob = Problem(
        dynamics="QUAD12", cost=cost,
        dyn_params=_f32([m, inertia, inertia, inertia, g], 8),
        x_init=_f32([0.1, 0.5, 0.5] + [0.0] * 9, MAX_STATE),
        x_lo=_f32([-INF, -INF, -INF, -1, -1, -INF, -1, -1, -1, -10, -10, -10], MAX_STATE),
        x_hi=_f32([INF, INF, INF, 1, 1, INF, 1, 1, 1, 10, 10, 10], MAX_STATE),
        u_lo=_f32([0, -0.5, -0.5, -0.5], MAX_CONTROL),
        u_hi=_f32([2 * m * g, 0.5, 0.5, 0.5], MAX_CONTROL),
        ws_lo=_f32([0, 0, 0], 3), ws_hi=_f32([1, 1, 1], 3),
        boxes=boxes, margin=float(np.float32(margin)),
        goal_center=_f32([0.9, 0.5, 0.5], 3), goal_radius=float(np.float32(0.05)),
    )
    prm = Params(dt=float(np.float32(0.005)), steps_min=steps[0], steps_max=steps[1],
                 grid=tuple(grid), vel_sign_bins=vel_sign_bins, n_select=n_select,
                 samples_per_node=samples, tree_cap=tree_cap, i_max=i_max, seed=seed)
    return Workload("quad12", prob, prm, iterations)


def _building_boxes(rng, n, start_xy, goal_xy, keep_out=0.2):
    boxes = []
    while len(boxes) < n:
        c = rng.uniform(0.0, 1.0, size=2)
        s = rng.uniform(0.03, 0.1, size=2)
        h = rng.uniform(0.2, 0.9)
        lo, hi = c - s / 2, c + s / 2
        bad = False
        for p in (start_xy, goal_xy):
            q = np.clip(p, lo, hi)
            if float(np.linalg.norm(q - p)) < keep_out:
                bad = True
        if bad:
            continue
        boxes.append([lo[0], lo[1], 0.0, hi[0], hi[1], h])
    return np.asarray(boxes, dtype=np.float32).reshape(n, 6)


def dubins6_workload(seed: int = 0, *, n_boxes: int = 200, n_select: int = 8192,
                     samples: int = 32, tree_cap: int = 1 << 22, grid=(32, 32, 16),
                     iterations: int = 200, i_max: int = 10, margin: float = 1e-4,
                     steps=(5, 30), cost: str = "PATH_LENGTH") -> Workload:
    """6D Dubins-airplane-like model: x, y, z, yaw, pitch, speed.

    Start (0.05, 0.05, 0.7) heading pi/4 at speed 0.5, goal ball r = 0.05 at
    (0.95, 0.95, 0.7).  No building footprint comes within 0.2 of the start or
    goal in xy: the airplane's turning radius is at least 0.2, so a tighter
    keep-out boxes it in against the workspace walls at the corner start."""
    start = np.array([0.05, 0.05])
    goal = np.array([0.95, 0.95])
    rng = _rng(seed, 0xDB6)
    boxes = _building_boxes(rng, n_boxes, start, goal)
    quarter_pi = math.pi / 4
    prob = Problem(
        dynamics="DUBINS6", cost=cost,
        dyn_params=_f32([], 8),
        x_init=_f32([0.05, 0.05, 0.7, quarter_pi, 0.0, 0.5], MAX_STATE),
        x_lo=_f32([-INF, -INF, -INF, -INF, -quarter_pi, 0.2], MAX_STATE),
        x_hi=_f32([INF, INF, INF, INF, quarter_pi, 1.0], MAX_STATE),
        u_lo=_f32([-1.0, -0.5, -0.5], MAX_CONTROL), u_hi=_f32([1.0, 0.5, 0.5], MAX_CONTROL),
        ws_lo=_f32([0, 0, 0], 3), ws_hi=_f32([1, 1, 1], 3),
        boxes=boxes, margin=float(np.float32(margin)),
        goal_center=_f32([0.95, 0.95, 0.7], 3), goal_radius=float(np.float32(0.05)),
    )
    prm = Params(dt=float(np.float32(0.01)), steps_min=steps[0], steps_max=steps[1],
                 grid=tuple(grid), vel_sign_bins=0, n_select=n_select,
                 samples_per_node=samples, tree_cap=tree_cap, i_max=i_max, seed=seed)
    return Workload("dubins6", prob, prm, iterations)


def _start_goal(rng, min_dist=0.6, lo=0.1, hi=0.9):
    while True:
        a, b = rng.uniform(lo, hi, size=3), rng.uniform(lo, hi, size=3)
        if np.linalg.norm(a - b) >= min_dist:
            return a, b


def batch_workloads(seed: int = 0, n_queries: int = 256, *, samples=None, iterations: int = 100,
                    margin: float = 1e-4) -> list:
    """Independent queries for the batched form: half double integrators
    (even query index) and half quadrotors (odd), each with its own seeded
    scene of U{4..256} boxes (centres U[0.1,0.9]^3, sides U[0.03,0.1]^3), a
    start and goal ball (r = 0.05) drawn in [0.1,0.9]^3 at least 0.6 apart, a
    tree capacity 2^U{10..18} and U{64..4096} nodes per iteration, clipped so
    that one iteration's candidates fit in half the tree.  `samples` maps
    "DI6" / "QUAD12" to the samples per node (default 8 / 16).  Query q has
    query_id q and planner seed `seed`."""
    samples = dict({"DI6": 8, "QUAD12": 16}, **(samples or {}))
    out = []
    for q in range(n_queries):
        rng = np.random.default_rng(np.random.SeedSequence([int(seed) & 0xFFFFFFFF, 0xBA7, q]))
        quad = q % 2 == 1
        dyn = "QUAD12" if quad else "DI6"
        start, goal = _start_goal(rng)
        n_boxes = int(rng.integers(4, 257))
        boxes = _random_boxes(rng, n_boxes, 0.1, 0.9, 0.03, 0.1, start, goal, 0.05)
        cap = 1 << int(rng.integers(10, 19))
        k = int(samples[dyn])
        n_select = int(np.exp(rng.uniform(np.log(64), np.log(4096))))
        n_select = max(1, min(n_select, (cap // 2) // k))
        if quad:
            m, inertia, g = 1.0, 0.01, 9.81
            prob = Problem(
                dynamics="QUAD12", cost="TIME",
                dyn_params=_f32([m, inertia, inertia, inertia, g], 8),
                x_init=_f32(list(start) + [0.0] * 9, MAX_STATE),
                x_lo=_f32([-INF, -INF, -INF, -1, -1, -INF, -1, -1, -1, -10, -10, -10], MAX_STATE),
                x_hi=_f32([INF, INF, INF, 1, 1, INF, 1, 1, 1, 10, 10, 10], MAX_STATE),
                u_lo=_f32([0, -0.5, -0.5, -0.5], MAX_CONTROL),
                u_hi=_f32([2 * m * g, 0.5, 0.5, 0.5], MAX_CONTROL),
                ws_lo=_f32([0, 0, 0], 3), ws_hi=_f32([1, 1, 1], 3),
                boxes=boxes, margin=float(np.float32(margin)),
                goal_center=_f32(goal, 3), goal_radius=float(np.float32(0.05)))
            prm = Params(dt=float(np.float32(0.005)), steps_min=5, steps_max=60, grid=(16, 16, 16),
                         vel_sign_bins=1, n_select=n_select, samples_per_node=k, tree_cap=cap,
                         i_max=10, seed=seed, query_id=q)
        else:
            prob = Problem(
                dynamics="DI6", cost="TIME",
                dyn_params=_f32([], 8),
                x_init=_f32(list(start) + [0.0] * 3, MAX_STATE),
                x_lo=_f32([-INF, -INF, -INF, -1, -1, -1], MAX_STATE),
                x_hi=_f32([INF, INF, INF, 1, 1, 1], MAX_STATE),
                u_lo=_f32([-1, -1, -1], MAX_CONTROL), u_hi=_f32([1, 1, 1], MAX_CONTROL),
                ws_lo=_f32([0, 0, 0], 3), ws_hi=_f32([1, 1, 1], 3),
                boxes=boxes, margin=float(np.float32(margin)),
                goal_center=_f32(goal, 3), goal_radius=float(np.float32(0.05)))
            prm = Params(dt=float(np.float32(0.01)), steps_min=5, steps_max=30, grid=(30, 30, 30),
                         vel_sign_bins=0, n_select=n_select, samples_per_node=k, tree_cap=cap,
                         i_max=10, seed=seed, query_id=q)
        out.append(Workload(f"batch/{dyn.lower()}/{q}", prob, prm, iterations))
    return out


@dataclasses.dataclass
class DiffBatch:
    """Edges for the differentiable rollout: the quadrotor scene (problem), its
    step size, and per edge a start state x0 (E x 12), 4 control segments u
    (E x 16, segment-major) and a step count n (E)."""
    problem: Problem
    dt: float
    x0: np.ndarray
    u: np.ndarray
    n: np.ndarray


def diff_workload(seed: int = 0, n_edges: int = 65536, steps=(20, 40)) -> DiffBatch:
    """Quadrotor edges in the 64-box wall scene of quad12_workload: starts
    uniform over the start side (x in [0.05, 0.45], y, z in [0.05, 0.95]) with
    small attitudes (|roll|, |pitch| <= 0.2), any yaw, velocities in
    [-0.5, 0.5] and body rates in [-1, 1]; each of the 4 control segments
    uniform in the control box; n uniform in steps, dt = 0.005."""
    w = quad12_workload(seed)
    rng = _rng(seed, 0xD1F)
    E = int(n_edges)
    x0 = np.zeros((E, 12), np.float32)
    x0[:, 0] = rng.uniform(0.05, 0.45, E)
    x0[:, 1:3] = rng.uniform(0.05, 0.95, (E, 2))
    x0[:, 3:5] = rng.uniform(-0.2, 0.2, (E, 2))
    x0[:, 5] = rng.uniform(-np.pi, np.pi, E)
    x0[:, 6:9] = rng.uniform(-0.5, 0.5, (E, 3))
    x0[:, 9:12] = rng.uniform(-1.0, 1.0, (E, 3))
    lo = np.asarray(w.problem.u_lo[:4], np.float32)
    hi = np.asarray(w.problem.u_hi[:4], np.float32)
    u = (lo + (hi - lo) * rng.uniform(0.0, 1.0, (E, 4, 4))).astype(np.float32).reshape(E, 16)
    n = rng.integers(steps[0], steps[1] + 1, E).astype(np.int32)
    return DiffBatch(w.problem, w.params.dt, x0, u, n)


# The uncapped form at the paper's large-delta sizes (App. B): every active
# node is expanded, the candidate buffer holds t_e slots shared out as
# lambda = floor(t_e / |V_A|), the tree holds t_e nodes, and the regions number
# about the paper's 27,000 / 52,000 / 100,000 (30^3; 40 x 40 x 32 = 51,200;
# 23^3 x 8 velocity-sign classes = 97,336).
PAPER_SIZES = {
    "di6": dict(n_select=100_000, samples=0, tree_cap=100_000, grid=(30, 30, 30)),
    "dubins6": dict(n_select=300_000, samples=0, tree_cap=300_000, grid=(40, 40, 32)),
    "quad12": dict(n_select=1_000_000, samples=0, tree_cap=1_000_000, grid=(23, 23, 23)),
}


def _paper(name):
    def make(seed: int = 0, **overrides) -> Workload:
        w = WORKLOADS[name](seed, **dict(PAPER_SIZES[name], **overrides))
        w.name = name + "_paper"
        return w
    return make


# The paper's small-delta sizes (App. B): t_e = 10^8 slots and nodes with about
# 10^7 regions for every system (215^3; 250 x 250 x 160; 108^3 x 8 velocity-sign
# classes).  About 21 GB of device memory per query.
PAPER_SMALL_SIZES = {
    "di6": dict(n_select=100_000_000, samples=0, tree_cap=100_000_000, grid=(215, 215, 215)),
    "dubins6": dict(n_select=100_000_000, samples=0, tree_cap=100_000_000, grid=(250, 250, 160)),
    "quad12": dict(n_select=100_000_000, samples=0, tree_cap=100_000_000, grid=(108, 108, 108)),
}


def _paper_small(name):
    def make(seed: int = 0, **overrides) -> Workload:
        w = WORKLOADS[name](seed, **dict(PAPER_SMALL_SIZES[name], **overrides))
        w.name = name + "_paper_small"
        return w
    return make


WORKLOADS = {"di6": di6_workload, "quad12": quad12_workload, "dubins6": dubins6_workload}
WORKLOADS.update({n + "_paper": _paper(n) for n in ("di6", "quad12", "dubins6")})
WORKLOADS.update({n + "_paper_small": _paper_small(n) for n in ("di6", "quad12", "dubins6")})


def make_workload(name: str, seed: int = 0, **overrides) -> Workload:
    return WORKLOADS[name](seed, **overrides)


def small_overrides(name: str) -> Dict[str, object]:
    """Reduced sizes that the oracle finishes in seconds yet still span several
    GPU tiles and leave a ragged tail (slot counts that are not multiples of 256)."""
    return {
        "di6": dict(n_select=100, samples=7, tree_cap=1 << 14),
        "quad12": dict(n_select=90, samples=9, tree_cap=1 << 15, grid=(8, 8, 8)),
        "dubins6": dict(n_select=120, samples=5, tree_cap=1 << 15, grid=(16, 16, 8)),
    }[name]


def describe(w: Workload, extra: Optional[dict] = None) -> dict:
    p, q = w.problem, w.params
    d = {
        "workload": w.name, "dynamics": p.dynamics, "cost": p.cost, "n_boxes": p.n_boxes,
        "n_select": q.n_select, "samples_per_node": q.samples_per_node,
        "edges_per_iteration": q.n_slots, "n_cells": q.n_cells, "tree_cap": q.tree_cap,
        "dt": q.dt, "steps": [q.steps_min, q.steps_max], "iterations": w.iterations,
        "seed": q.seed,
    }
    if extra:
        d.update(extra)
    return d
