"""ctypes wrapper of the float64 reference (kpx_oracle.c).

TEST INFRASTRUCTURE: imported only by tests/, the smoke check and the CPU
baseline leg of bench.py.  The planner package never imports this module.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kpx_oracle.c")
SRC_DIFF = os.path.join(HERE, "kpx_oracle_diff.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")  # the same source with OpenMP (CPU timing only)

MAX_STATE = 12
MAX_CONTROL = 4
ACTIVE, INACTIVE, TERMINAL = 0, 1, 2
OK, FULL, ERR_ARG, ERR_INVALID_START = 0, 1, -1, -2
FLAG_BOX, FLAG_WORKSPACE, FLAG_BOUND, FLAG_CELL, FLAG_VSIGN, FLAG_GOAL, FLAG_TIE = (
    1, 2, 4, 8, 16, 32, 64)
DYN = {"DI6": 0, "QUAD12": 1, "DUBINS6": 2}
COST = {"TIME": 0, "PATH_LENGTH": 1}

_f32p = C.POINTER(C.c_float)
_f64p = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_u8p = C.POINTER(C.c_uint8)
_u32p = C.POINTER(C.c_uint32)


class ProblemC(C.Structure):
    _fields_ = [
        ("dynamics", C.c_int32), ("cost", C.c_int32), ("dyn_params", C.c_float * 8),
        ("x_init", C.c_float * MAX_STATE), ("x_lo", C.c_float * MAX_STATE),
        ("x_hi", C.c_float * MAX_STATE), ("u_lo", C.c_float * MAX_CONTROL),
        ("u_hi", C.c_float * MAX_CONTROL), ("ws_lo", C.c_float * 3), ("ws_hi", C.c_float * 3),
        ("boxes", _f32p), ("n_boxes", C.c_int32), ("margin", C.c_float),
        ("goal_center", C.c_float * 3), ("goal_radius", C.c_float), ("dt", C.c_float),
        ("steps_min", C.c_int32), ("steps_max", C.c_int32), ("grid", C.c_int32 * 3),
        ("vel_sign_bins", C.c_int32), ("n_select", C.c_int32),
        ("samples_per_node", C.c_int32),
        ("tree_cap", C.c_int64), ("i_max", C.c_int32), ("seed", C.c_uint64),
        ("query_id", C.c_uint32), ("band", C.c_double),
        ("polish_steps", C.c_int32), ("polish_lr", C.c_double), ("polish_w_ctrl", C.c_double),
        ("polish_w_obst", C.c_double), ("polish_k_obst", C.c_double), ("polish_d_safe", C.c_double),
        ("polish_w_goal", C.c_double), ("polish_w_len", C.c_double), ("polish_goal_only", C.c_int32),
    ]


class TreeC(C.Structure):
    _fields_ = [
        ("cap", C.c_int64), ("n_tree", C.c_int64), ("x", _f64p), ("u", _f32p),
        ("steps", _i32p), ("parent", _i64p), ("cost", _f64p), ("cell", _i64p),
        ("status", _u8p), ("icount", _i32p), ("n_cells", C.c_int64), ("tbl_cost", _f64p),
        ("tbl_id", _i64p), ("cursor", C.c_int64), ("iter", C.c_int64), ("sol_cost", C.c_double),
        ("sol_id", C.c_int64), ("first_sol_iter", C.c_int64), ("full", C.c_int32),
        ("last_n_sel", C.c_int64), ("last_n_valid", C.c_int64), ("last_n_surv", C.c_int64),
    ]


class CandsC(C.Structure):
    _fields_ = [
        ("cap_slots", C.c_int64), ("n_slots", C.c_int64), ("parent", _i64p), ("u", _f32p),
        ("n", _i32p), ("xn", _f64p), ("valid", _u8p), ("first_invalid", _i32p),
        ("substeps", _i32p), ("flags", _u32p), ("cell", _i64p), ("cost", _f64p), ("goal", _u8p),
        ("survivor", _u8p), ("new_index", _i64p), ("polished", _u8p),
        ("substeps_total", C.c_int64), ("k", C.c_int64),
    ]


class HintsC(C.Structure):
    _fields_ = [("first_invalid", _i32p), ("cell", _i64p), ("goal", _u8p), ("survivor", _u8p),
                ("polish_first_invalid", _i32p), ("polish_cell", _i64p), ("polish_goal", _u8p),
                ("polish_accepted", _u8p)]


class EdgeC(C.Structure):
    _fields_ = [("xn", C.c_double * MAX_STATE), ("length", C.c_double),
                ("first_invalid", C.c_int32), ("substeps", C.c_int32), ("flags", C.c_uint32)]


class VerifyC(C.Structure):
    _fields_ = [
        ("ok", C.c_int32), ("starts_at_init", C.c_int32), ("collision_free", C.c_int32),
        ("within_bounds", C.c_int32), ("reaches_goal", C.c_int32), ("cost_ok", C.c_int32),
        ("first_bad_edge", C.c_int32), ("first_bad_substep", C.c_int32), ("cost", C.c_double),
        ("min_clearance", C.c_double), ("max_gap", C.c_double), ("goal_distance", C.c_double),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (strict IEEE float64, no fast-math), and the
    same source with OpenMP for the CPU-baseline timing."""
    deps = [SRC, SRC_DIFF, os.path.join(HERE, "kpx_oracle.h"), os.path.join(HERE, "kpx_oracle_diff.h")]
    for out, extra in ((LIB, ["-Wno-unknown-pragmas"]), (LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < max(map(os.path.getmtime, deps)):
            tmp = out + ".tmp"
            subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                                   "-ffp-contract=off", "-Wall", "-Wextra", *extra, "-o", tmp, SRC,
                                   SRC_DIFF, "-lm"])
            os.replace(tmp, out)
    return LIB


_lib = None
_lib_omp = None


def lib_threads():
    """The OpenMP build, for timing the oracle on every host core (its step
    gives the same results as the plain build's)."""
    global _lib_omp
    if _lib_omp is None:
        build()
        L = C.CDLL(LIB_OMP)
        L.ora_step.argtypes = lib().ora_step.argtypes
        L.ora_step.restype = C.c_int
        L.ora_threads.restype = C.c_int
        _lib_omp = L
    return _lib_omp


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        L.ora_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.ora_philox_many.argtypes = [_u32p, C.c_int64, _u32p]
        L.ora_sample.argtypes = [C.POINTER(ProblemC), C.c_uint32, C.c_uint32, _f32p, _i32p]
        L.ora_deriv.argtypes = [C.POINTER(ProblemC), _f64p, _f64p, _f64p]
        L.ora_rk4_step.argtypes = [C.POINTER(ProblemC), _f64p, _f64p, C.c_double]
        L.ora_integrate.argtypes = [C.POINTER(ProblemC), _f64p, _f64p, C.c_int32, C.c_double, _f64p]
        L.ora_point_status.argtypes = [C.POINTER(ProblemC), _f64p, C.c_double, C.c_double, _u32p]
        L.ora_point_status.restype = C.c_int
        L.ora_cell_of.argtypes = [C.POINTER(ProblemC), _f64p, _i64p, _u32p]
        L.ora_cell_of.restype = C.c_int64
        L.ora_goal_test.argtypes = [C.POINTER(ProblemC), _f64p, C.c_double, _u8p, _u32p]
        L.ora_goal_test.restype = C.c_int
        L.ora_propagate_edge.argtypes = [C.POINTER(ProblemC), _f64p, _f32p, C.c_int32, C.c_int32,
                                         C.POINTER(EdgeC)]
        L.ora_exclusive_scan.argtypes = [_u8p, C.c_int64, _i64p]
        L.ora_graph_search.argtypes = [_u8p, _i64p, C.c_int64, _i64p]
        L.ora_graph_search.restype = C.c_int64
        L.ora_init.argtypes = [C.POINTER(ProblemC), C.POINTER(TreeC)]
        L.ora_init.restype = C.c_int
        L.ora_select.argtypes = [C.POINTER(ProblemC), C.POINTER(TreeC), _i64p, _i64p]
        L.ora_select.restype = C.c_int64
        L.ora_prune.argtypes = [C.POINTER(ProblemC), C.POINTER(TreeC)]
        L.ora_step.argtypes = [C.POINTER(ProblemC), C.POINTER(TreeC), C.POINTER(CandsC),
                               C.POINTER(HintsC)]
        L.ora_refine.argtypes = [C.POINTER(ProblemC), C.POINTER(TreeC), C.c_int32, _i64p]
        L.ora_step.restype = C.c_int
        L.ora_verify.argtypes = [C.POINTER(ProblemC), C.c_int32, _f32p, _i32p, _f32p, C.c_double,
                                 C.POINTER(VerifyC)]
        L.ora_verify.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ct)


class Problem:
    """Oracle view of a problem + parameters (keeps the box array alive)."""

    def __init__(self, problem, params, band: float = 1e-5, polish: Optional[dict] = None):
        self.problem, self.params = problem, params
        self.boxes = np.ascontiguousarray(problem.boxes, dtype=np.float32).reshape(-1, 6)
        s = ProblemC()
        s.dynamics = DYN[problem.dynamics]
        s.cost = COST[problem.cost]
        for name in ("dyn_params", "x_init", "x_lo", "x_hi", "u_lo", "u_hi", "ws_lo", "ws_hi",
                     "goal_center"):
            arr = np.asarray(getattr(problem, name), dtype=np.float32)
            getattr(s, name)[:] = [float(v) for v in arr]
        s.boxes = _ptr(self.boxes, _f32p) if self.boxes.size else None
        s.n_boxes = self.boxes.shape[0]
        s.margin = problem.margin
        s.goal_radius = problem.goal_radius
        s.dt = params.dt
        s.steps_min, s.steps_max = params.steps_min, params.steps_max
        s.grid[:] = list(params.grid)
        s.vel_sign_bins = params.vel_sign_bins
        s.n_select, s.samples_per_node = params.n_select, params.samples_per_node
        s.tree_cap = params.tree_cap
        s.i_max = params.i_max
        s.seed = params.seed
        s.query_id = params.query_id
        s.band = band
        if polish:  # float32 values widened, as the device receives them
            f = lambda v: float(np.float32(v))  # noqa: E731
            s.polish_steps = int(polish.get("steps", 3))
            s.polish_lr = f(polish.get("lr", 0.01))
            s.polish_w_ctrl = f(polish.get("w_ctrl", 0.1))
            s.polish_w_obst = f(polish.get("w_obst", 1.0))
            s.polish_k_obst = f(polish.get("k_obst", 50.0))
            s.polish_d_safe = f(polish.get("d_safe", 0.02))
            s.polish_w_goal = f(polish.get("w_goal", 1.0))
            s.polish_w_len = f(polish.get("w_len", 0.0))
            s.polish_goal_only = int(bool(polish.get("goal_only", False)))
        self.c = s
        self.d = {"DI6": 6, "QUAD12": 12, "DUBINS6": 6}[problem.dynamics]
        self.m = {"DI6": 3, "QUAD12": 4, "DUBINS6": 3}[problem.dynamics]
        self.n_cells = params.n_cells

    @property
    def ref(self):
        return C.byref(self.c)


def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().ora_philox4x32_10(_ptr(c, _u32p), _ptr(k, _u32p), _ptr(out, _u32p))
    return out


def philox_many(counter_key) -> np.ndarray:
    ck = np.ascontiguousarray(counter_key, dtype=np.uint32).reshape(-1, 6)
    out = np.zeros((ck.shape[0], 4), dtype=np.uint32)
    lib().ora_philox_many(_ptr(ck, _u32p), ck.shape[0], _ptr(out, _u32p))
    return out


def sample(P: Problem, it: int, slot: int):
    u = np.zeros(MAX_CONTROL, dtype=np.float32)
    n = np.zeros(1, dtype=np.int32)
    lib().ora_sample(P.ref, it, slot, _ptr(u, _f32p), _ptr(n, _i32p))
    return u, int(n[0])


def deriv(P: Problem, z, u) -> np.ndarray:
    zz = np.zeros(MAX_STATE + 1)
    zz[: len(z)] = z
    uu = np.zeros(MAX_CONTROL)
    uu[: len(u)] = u
    out = np.zeros(MAX_STATE + 1)
    lib().ora_deriv(P.ref, _ptr(zz, _f64p), _ptr(uu, _f64p), _ptr(out, _f64p))
    return out[: P.d + 1]


def integrate(P: Problem, x0, u, n: int, h: Optional[float] = None) -> np.ndarray:
    """n RK4 steps of size h (default dt); returns (state, path length)."""
    x = np.zeros(MAX_STATE)
    x[: P.d] = np.asarray(x0, dtype=np.float64)[: P.d]
    uu = np.zeros(MAX_CONTROL)
    uu[: len(u)] = u
    out = np.zeros(MAX_STATE + 1)
    lib().ora_integrate(P.ref, _ptr(x, _f64p), _ptr(uu, _f64p), n,
                        float(P.params.dt if h is None else h), _ptr(out, _f64p))
    return out[: P.d + 1]


def point_status(P: Problem, x, margin: Optional[float] = None, band: float = 0.0):
    xx = np.zeros(MAX_STATE)
    xx[: len(x)] = x
    fl = np.zeros(1, dtype=np.uint32)
    m = P.problem.margin if margin is None else margin
    st = lib().ora_point_status(P.ref, _ptr(xx, _f64p), float(m), float(band), _ptr(fl, _u32p))
    return bool(st & 1), bool(st & 2), int(fl[0])


def cell_of(P: Problem, x, hint: Optional[int] = None):
    xx = np.zeros(MAX_STATE)
    xx[: len(x)] = x
    fl = np.zeros(1, dtype=np.uint32)
    h = np.array([hint], dtype=np.int64) if hint is not None else None
    c = lib().ora_cell_of(P.ref, _ptr(xx, _f64p), _ptr(h, _i64p) if h is not None else None,
                          _ptr(fl, _u32p))
    return int(c), int(fl[0])


def goal_test(P: Problem, x, radius: Optional[float] = None):
    xx = np.zeros(MAX_STATE)
    xx[: len(x)] = x
    fl = np.zeros(1, dtype=np.uint32)
    r = (P.problem.goal_radius - P.problem.margin) if radius is None else radius
    return bool(lib().ora_goal_test(P.ref, _ptr(xx, _f64p), float(r), None, _ptr(fl, _u32p))), int(fl[0])


def propagate_edge(P: Problem, x0, u, n: int, hint_first_invalid: int = -1) -> dict:
    x = np.zeros(MAX_STATE)
    x[: P.d] = np.asarray(x0, dtype=np.float64)[: P.d]
    uu = np.zeros(MAX_CONTROL, dtype=np.float32)
    uu[: len(u)] = u
    e = EdgeC()
    lib().ora_propagate_edge(P.ref, _ptr(x, _f64p), _ptr(uu, _f32p), n, hint_first_invalid,
                             C.byref(e))
    return {"xn": np.array(e.xn[: P.d]), "length": e.length, "first_invalid": e.first_invalid,
            "substeps": e.substeps, "flags": e.flags}


def exclusive_scan(mask) -> np.ndarray:
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    S = np.zeros(max(1, m.size), dtype=np.int64)
    lib().ora_exclusive_scan(_ptr(m, _u8p), m.size, _ptr(S, _i64p))
    return S[: m.size]


def graph_search(mask, S):
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    s = np.ascontiguousarray(S, dtype=np.int64)
    I = np.full(max(1, m.size), -1, dtype=np.int64)
    count = lib().ora_graph_search(_ptr(m, _u8p), _ptr(s, _i64p), m.size, _ptr(I, _i64p))
    return I[: m.size], int(count)


class Cands:
    def __init__(self, cap_slots: int):
        n = max(1, int(cap_slots))
        self.parent = np.zeros(n, np.int64)
        self.u = np.zeros((n, MAX_CONTROL), np.float32)
        self.n = np.zeros(n, np.int32)
        self.xn = np.zeros((n, MAX_STATE), np.float64)
        self.valid = np.zeros(n, np.uint8)
        self.first_invalid = np.zeros(n, np.int32)
        self.substeps = np.zeros(n, np.int32)
        self.flags = np.zeros(n, np.uint32)
        self.cell = np.zeros(n, np.int64)
        self.cost = np.zeros(n, np.float64)
        self.goal = np.zeros(n, np.uint8)
        self.survivor = np.zeros(n, np.uint8)
        self.new_index = np.zeros(n, np.int64)
        self.polished = np.zeros(n, np.uint8)
        s = CandsC()
        s.cap_slots = int(cap_slots)
        for name, ct in (("parent", _i64p), ("u", _f32p), ("n", _i32p), ("xn", _f64p),
                         ("valid", _u8p), ("first_invalid", _i32p), ("substeps", _i32p),
                         ("flags", _u32p), ("cell", _i64p), ("cost", _f64p), ("goal", _u8p),
                         ("survivor", _u8p), ("new_index", _i64p), ("polished", _u8p)):
            setattr(s, name, _ptr(getattr(self, name), ct))
        self.c = s

    @property
    def n_slots(self) -> int:
        return int(self.c.n_slots)

    @property
    def substeps_total(self) -> int:
        return int(self.c.substeps_total)

    @property
    def k(self) -> int:
        """Samples per selected node in the last step."""
        return int(self.c.k)

    def view(self) -> dict:
        k = self.n_slots
        return {name: getattr(self, name)[:k].copy() for name in (
            "parent", "u", "n", "xn", "valid", "first_invalid", "substeps", "flags", "cell",
            "cost", "goal", "survivor", "new_index", "polished")}


class Tree:
    """The oracle's float64 tree (caller-owned numpy storage)."""

    def __init__(self, P: Problem, cap: Optional[int] = None, cells_cap: Optional[int] = None):
        self.P = P
        cap = int(P.params.tree_cap if cap is None else cap)
        nc = max(P.n_cells, int(cells_cap or 0))  # region arrays; refinement may grow the count
        self.x = np.zeros((cap, MAX_STATE), np.float64)
        self.u = np.zeros((cap, MAX_CONTROL), np.float32)
        self.steps = np.zeros(cap, np.int32)
        self.parent = np.full(cap, -1, np.int64)
        self.cost = np.zeros(cap, np.float64)
        self.cell = np.zeros(cap, np.int64)
        self.status = np.full(cap, TERMINAL, np.uint8)
        self.icount = np.zeros(cap, np.int32)
        self.tbl_cost = np.full(nc, np.inf, np.float64)
        self.tbl_id = np.full(nc, -1, np.int64)
        s = TreeC()
        s.cap = cap
        s.n_cells = P.n_cells
        for name, ct in (("x", _f64p), ("u", _f32p), ("steps", _i32p), ("parent", _i64p),
                         ("cost", _f64p), ("cell", _i64p), ("status", _u8p), ("icount", _i32p),
                         ("tbl_cost", _f64p), ("tbl_id", _i64p)):
            setattr(s, name, _ptr(getattr(self, name), ct))
        s.sol_cost = np.inf
        s.sol_id = -1
        s.first_sol_iter = -1
        self.c = s
        self.cands = Cands(P.params.n_slots)

    def init(self) -> int:
        return lib().ora_init(self.P.ref, C.byref(self.c))

    @property
    def n_tree(self) -> int:
        return int(self.c.n_tree)

    def step(self, hints: Optional[dict] = None, threaded: bool = False) -> int:
        h = None
        keep = []
        if hints is not None:
            hc = HintsC()
            for name, dt, ct in (("first_invalid", np.int32, _i32p), ("cell", np.int64, _i64p),
                                 ("goal", np.uint8, _u8p), ("survivor", np.uint8, _u8p),
                                 ("polish_first_invalid", np.int32, _i32p),
                                 ("polish_cell", np.int64, _i64p), ("polish_goal", np.uint8, _u8p),
                                 ("polish_accepted", np.uint8, _u8p)):
                if hints.get(name) is not None:
                    a = np.ascontiguousarray(hints[name], dtype=dt)
                    keep.append(a)
                    setattr(hc, name, _ptr(a, ct))
            h = C.byref(hc)
        L = lib_threads() if threaded else lib()
        return L.ora_step(self.P.ref, C.byref(self.c), C.byref(self.cands.c), h)

    def refine(self, P_new: Problem, factor: int, hint_cell=None) -> int:
        """Adaptive decomposition: P_new is the problem with the refined grid
        (see ora_refine); hint_cell (optional, per node) is the other side's
        region of each node."""
        assert len(self.tbl_id) >= P_new.n_cells
        self.P = P_new
        h = None
        if hint_cell is not None:
            h = np.ascontiguousarray(hint_cell, dtype=np.int64)
        rc = lib().ora_refine(P_new.ref, C.byref(self.c), int(factor), _ptr(h, _i64p) if h is not None else None)
        self._keep_hint = h
        return rc

    def select(self):
        sel = np.zeros(max(1, self.P.params.n_select), np.int64)
        cur = np.zeros(1, np.int64)
        k = lib().ora_select(self.P.ref, C.byref(self.c), _ptr(sel, _i64p), _ptr(cur, _i64p))
        return sel[:k].copy(), int(cur[0])

    def prune(self):
        lib().ora_prune(self.P.ref, C.byref(self.c))

    def set_scalars(self, **kw):
        for k, v in kw.items():
            setattr(self.c, k, v)

    def scalars(self) -> dict:
        return {k: getattr(self.c, k) for k in ("n_tree", "cursor", "iter", "sol_cost", "sol_id",
                                                "first_sol_iter", "full", "last_n_sel",
                                                "last_n_valid", "last_n_surv")}

    def path_to(self, idx: int):
        """Edges from the root to node idx: (controls, steps, states)."""
        chain = []
        i = idx
        while i >= 0:
            chain.append(i)
            i = int(self.parent[i])
        chain = chain[::-1]
        ctrl = self.u[chain[1:]].astype(np.float32)
        steps = self.steps[chain[1:]].astype(np.int32)
        states = self.x[chain].astype(np.float32)
        return ctrl, steps, states


def verify(P: Problem, controls, steps, states=None, reported_cost: float = 0.0) -> dict:
    n = int(len(steps))
    ctrl = np.zeros((max(1, n), MAX_CONTROL), np.float32)
    c_in = np.asarray(controls, dtype=np.float32).reshape(n, -1) if n else np.zeros((0, 1))
    ctrl[:n, : c_in.shape[1]] = c_in
    st = np.ascontiguousarray(np.asarray(steps, dtype=np.int32).reshape(-1))
    if st.size == 0:
        st = np.zeros(1, np.int32)
    sp = None
    if states is not None:
        s_in = np.asarray(states, dtype=np.float32).reshape(n + 1, -1)
        sarr = np.zeros((n + 1, MAX_STATE), np.float32)
        sarr[:, : s_in.shape[1]] = s_in
        sp = sarr
    rep = VerifyC()
    lib().ora_verify(P.ref, n, _ptr(ctrl, _f32p), _ptr(st, _i32p),
                     _ptr(sp, _f32p) if sp is not None else None, float(reported_cost),
                     C.byref(rep))
    return {name: getattr(rep, name) for name, _ in VerifyC._fields_}


def run(P: Problem, iterations: int, on_step=None) -> Tree:
    """Free-running float64 planner from x_init (Alg. 1 with an iteration budget)."""
    T = Tree(P)
    rc = T.init()
    if rc != OK:
        raise RuntimeError(f"oracle init failed: {rc}")
    for _ in range(iterations):
        rc = T.step()
        if on_step is not None:
            on_step(T)
        if rc == FULL:
            break
    return T


# ---------------------------------------------------------------- differentiable rollout

class OradProblemC(C.Structure):
    _fields_ = [
        ("mass", C.c_double), ("jx", C.c_double), ("jy", C.c_double), ("jz", C.c_double),
        ("grav", C.c_double), ("dt", C.c_double), ("boxes", _f32p), ("n_boxes", C.c_int32),
        ("goal", C.c_double * 3), ("w_ctrl", C.c_double), ("w_obst", C.c_double),
        ("k_obst", C.c_double), ("d_safe", C.c_double), ("w_goal", C.c_double),
        ("w_len", C.c_double),
    ]


_dlib = None


def _diff_lib():
    global _dlib
    if _dlib is None:
        L = lib()
        pp = C.POINTER(OradProblemC)
        L.orad_segment.argtypes = [C.c_int32, C.c_int32]
        L.orad_segment.restype = C.c_int32
        L.orad_box_sd.argtypes = [_f32p, _f64p]
        L.orad_box_sd.restype = C.c_double
        L.orad_loss.argtypes = [pp, _f64p, _f64p, C.c_int32, _f64p]
        L.orad_loss.restype = C.c_double
        L.orad_grad.argtypes = [pp, _f64p, _f64p, C.c_int32, C.c_double, _f64p]
        L.orad_grad.restype = None
        L.orad_grad_tied.argtypes = [pp, _f64p, _f64p, C.c_int32, C.c_double, _f64p]
        L.orad_grad_tied.restype = None
        L.orad_first_invalid.argtypes = [pp, _f64p, _f64p, C.c_int32, _f64p, _f64p, _f64p, _f64p]
        L.orad_first_invalid.restype = C.c_int32
        _dlib = L
    return _dlib


class DiffProblem:
    """The scene and loss weights of the differentiable rollout (float32
    values widened, as everywhere in the oracle)."""

    def __init__(self, problem, dt, goal=None, w_ctrl=0.1, w_obst=1.0, k_obst=50.0, d_safe=0.02,
                 w_goal=1.0, w_len=0.0):
        f = lambda v: float(np.float32(v))  # noqa: E731
        self.problem = problem
        self.boxes = np.ascontiguousarray(problem.boxes, dtype=np.float32).reshape(-1, 6)
        s = OradProblemC()
        dp = problem.dyn_params
        s.mass, s.jx, s.jy, s.jz, s.grav = (f(dp[0]), f(dp[1]), f(dp[2]), f(dp[3]), f(dp[4]))
        s.dt = f(dt)
        s.boxes = _ptr(self.boxes, _f32p) if self.boxes.size else None
        s.n_boxes = self.boxes.shape[0]
        g = problem.goal_center if goal is None else goal
        s.goal = (C.c_double * 3)(*[f(v) for v in g[:3]])
        s.w_ctrl, s.w_obst, s.k_obst, s.d_safe, s.w_goal = (f(w_ctrl), f(w_obst), f(k_obst),
                                                            f(d_safe), f(w_goal))
        s.w_len = f(w_len)
        self.c = s
        self.ref = C.byref(s)


def diff_segment(k: int, n: int) -> int:
    return int(_diff_lib().orad_segment(int(k), int(n)))


def box_sd(box, p) -> float:
    b = np.ascontiguousarray(box, dtype=np.float32)
    q = np.ascontiguousarray(p, dtype=np.float64)
    return float(_diff_lib().orad_box_sd(_ptr(b, _f32p), _ptr(q, _f64p)))


def diff_loss(D, x0, u, n, states=False):
    x = np.ascontiguousarray(x0, dtype=np.float64)
    uu = np.ascontiguousarray(u, dtype=np.float64).reshape(16)
    st = np.zeros(((int(n) + 1), 12), np.float64) if states else None
    L = _diff_lib().orad_loss(D.ref, _ptr(x, _f64p), _ptr(uu, _f64p), int(n),
                              _ptr(st, _f64p) if states else None)
    return (L, st) if states else L


def diff_grad(D, x0, u, n, h=1e-20):
    x = np.ascontiguousarray(x0, dtype=np.float64)
    uu = np.ascontiguousarray(u, dtype=np.float64).reshape(16)
    g = np.zeros(16, np.float64)
    _diff_lib().orad_grad(D.ref, _ptr(x, _f64p), _ptr(uu, _f64p), int(n), float(h), _ptr(g, _f64p))
    return g


def diff_grad_tied(D, x0, u, n, h=1e-20):
    x = np.ascontiguousarray(x0, dtype=np.float64)
    uu = np.ascontiguousarray(u, dtype=np.float64).reshape(16)
    g = np.zeros(4, np.float64)
    _diff_lib().orad_grad_tied(D.ref, _ptr(x, _f64p), _ptr(uu, _f64p), int(n), float(h), _ptr(g, _f64p))
    return g


def diff_first_invalid(D, x0, u, n):
    p = D.problem
    x = np.ascontiguousarray(x0, dtype=np.float64)
    uu = np.ascontiguousarray(u, dtype=np.float64).reshape(16)
    lo = np.ascontiguousarray(np.asarray(p.x_lo, np.float64)[:12])
    hi = np.ascontiguousarray(np.asarray(p.x_hi, np.float64)[:12])
    wl = np.ascontiguousarray(np.asarray(p.ws_lo, np.float64)[:3])
    wh = np.ascontiguousarray(np.asarray(p.ws_hi, np.float64)[:3])
    return int(_diff_lib().orad_first_invalid(D.ref, _ptr(x, _f64p), _ptr(uu, _f64p), int(n),
                                              _ptr(lo, _f64p), _ptr(hi, _f64p), _ptr(wl, _f64p),
                                              _ptr(wh, _f64p)))
