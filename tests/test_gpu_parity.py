"""GPU parity of the HIP planner (through the C ABI) against the float64 oracle."""

import numpy as np
import pytest

import workloads as W
from workloads.scenes import small_overrides

from oracle import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kpx():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_02846_amd as K

    K.lib()
    return K


def _planner(kpx, w):
    return kpx.Planner(w.problem, w.params)


def test_device_philox_matches_oracle(kpx, ora):
    rng = np.random.default_rng(3)
    ck = rng.integers(0, 2**32, size=(1_000_000, 6), dtype=np.uint64).astype(np.uint32)
    ck[:1000, 1] = np.arange(1000)  # the sample contract's counters: (it, slot, query, block)
    ck[:1000, 0] = 7
    ck[:1000, 2:4] = 0
    dev = kpx.philox(ck)
    ref = ora.philox_many(ck)
    np.testing.assert_array_equal(dev, ref)


# sizes the oracle replays in seconds that still span several survivor tiles
# (2048 slots each) and several propagate blocks (256), with ragged tails
LOCKSTEP = {
    "di6": (dict(n_select=300, samples=9, tree_cap=1 << 16), 40),
    "di6_path": (dict(n_select=300, samples=9, tree_cap=1 << 16, cost="PATH_LENGTH"), 30),
    "quad12": (dict(n_select=260, samples=9, tree_cap=1 << 16, grid=(8, 8, 8)), 25),
    "dubins6": (dict(n_select=230, samples=11, tree_cap=1 << 16, grid=(16, 16, 8)), 25),
    "quad12_path": (dict(n_select=260, samples=9, tree_cap=1 << 16, grid=(8, 8, 8), cost="PATH_LENGTH"), 20),
    "dubins6_path": (dict(n_select=230, samples=11, tree_cap=1 << 16, grid=(16, 16, 8), cost="PATH_LENGTH"), 20),
}


@pytest.mark.parametrize("case", sorted(LOCKSTEP))
def test_lockstep_iterations(kpx, ora, case):
    kw, iters = LOCKSTEP[case]
    name = case.split("_")[0]
    w = W.make_workload(name, 5, **kw)
    P = ora.Problem(w.problem, w.params)
    pl = _planner(kpx, w)
    rep = parity.lockstep(ora, P, pl, iters)
    print(case, rep)
    assert rep["iterations"] == iters
    assert rep["valid"] > 0
    pl.close()


def test_lockstep_small_configs_from_later_iterations(kpx, ora):
    """Run ahead without checking, then check: exercises larger trees, dormant
    nodes, reactivation and a solution already present."""
    w = W.make_workload("di6", 11, n_select=256, samples=8, i_max=2)
    P = ora.Problem(w.problem, w.params)
    pl = _planner(kpx, w)
    pl.iterate(60)
    pl.sync()
    snap = pl.snapshot()
    st = snap["status"]
    assert (st == kpx.INACTIVE).any() and (st == kpx.TERMINAL).any()
    rep = parity.lockstep(ora, P, pl, 15)
    assert rep["iterations"] == 15
    pl.close()


@pytest.mark.parametrize("name", ["di6", "quad12", "dubins6"])
def test_same_seed_same_tree(kpx, name):
    kw = small_overrides(name)
    trees = []
    for _ in range(2):
        w = W.make_workload(name, 2, **kw)
        pl = _planner(kpx, w)
        pl.iterate(30)
        trees.append(pl.snapshot())
        pl.close()
    a, b = trees
    for k in ("state", "control", "steps", "parent", "cost", "cell", "status", "icount", "cell_table"):
        np.testing.assert_array_equal(a[k], b[k])
    assert a["counters"] == b["counters"]


@pytest.mark.parametrize("name,kw,cost_first", [
    ("quad12", {}, False),                        # the benchmark shape, 4096 x 32 slots
    ("quad12", dict(cost="PATH_LENGTH"), False),
    ("quad12", {}, True),
    ("di6", {}, False),
    ("dubins6", {}, False),
])
def test_recording_leaves_the_tree_unchanged(kpx, name, kw, cost_first):
    """With every slot recorded (the record the lockstep tests replay) each
    slot writes its candidate record; otherwise only the slots that take a
    region's atomic minimum write theirs.  Both must grow the same tree."""
    trees = []
    for record in (True, False):
        w = W.make_workload(name, 4, **kw)
        pl = _planner(kpx, w)
        pl.set_dump(record)
        if cost_first:
            pl.set_cost_first(True)
        pl.iterate(60)
        trees.append(pl.snapshot())
        pl.close()
    a, b = trees
    assert a["counters"]["n_tree"] > 1000, a["counters"]
    for k in ("state", "control", "steps", "parent", "cost", "cell", "status", "icount", "cell_table"):
        np.testing.assert_array_equal(a[k], b[k])
    assert a["counters"] == b["counters"]


def test_double_integrator_solution_verifies(kpx, ora):
    w = W.make_workload("di6", 0)  # full size: 256 nodes x 8 samples
    P = ora.Problem(w.problem, w.params)
    pl = _planner(kpx, w)
    pl.iterate(w.iterations)
    sol = pl.solution()
    assert sol["found"], pl.counters()
    rep = ora.verify(P, sol["controls"], sol["steps"], sol["states"], float(sol["cost_field"]))
    assert rep["ok"], rep
    assert abs(sol["cost"] - sol["cost_field"] * w.params.dt) < 1e-9
    pl.close()


def test_stats_ring_and_timing(kpx):
    w = W.make_workload("di6", 1, **small_overrides("di6"))
    pl = _planner(kpx, w)
    pl.set_timing(True)
    pl.iterate(20)
    ms, launches = pl.read_timing()
    assert launches == [20, 20, 20, 20] and all(t > 0 for t in ms)
    st = pl.stats(0, 20)
    c = pl.counters()
    assert st["iteration"].tolist() == list(range(20))
    assert st["n_tree"][-1] == c["n_tree"]
    assert np.all(np.diff(st["n_tree"]) == st["n_survivors"][1:])
    assert np.all(st["t_end"] >= st["t_begin"])
    assert pl.clock_rate_khz() > 0
    # the regions a tree node kept through propagate, plus those this
    # iteration's survivors took, are the regions owned after it
    for _ in range(3):
        pl.iterate(1)
        c = pl.counters()
        r = pl.stats(int(c["iteration"]) - 1, 1)[0]
        owned = int((pl.snapshot()["cell_table"] != np.uint64(0xFFFFFFFFFFFFFFFF)).sum())
        assert int(r["n_live"]) + int(r["n_survivors"]) == owned, (r, owned)
    pl.set_timing(1)  # propagate only
    pl.iterate(5)
    ms, launches = pl.read_timing()
    assert launches == [5, 0, 0, 0] and ms[0] > 0 and ms[1:] == [0.0, 0.0, 0.0]
    pl.set_timing(15, every=4)  # iterations 0, 4, 8 of the next 10
    pl.iterate(10)
    ms, launches = pl.read_timing()
    assert launches == [3, 3, 3, 3] and all(t > 0 for t in ms)
    with pytest.raises(kpx.KPXError):
        pl.set_timing(16)
    with pytest.raises(kpx.KPXError):
        pl.set_timing(1, every=0)
    pl.close()


def test_timing_leaves_out_iterations_after_the_tree_filled(kpx):
    """Iterations enqueued after the tree filled return at once: their
    launches are not counted, so launches match the iterations that ran."""
    w = W.make_workload("di6_paper", 0)  # 10^5 slots into a 10^5-node tree: full within ~25 iterations
    pl = _planner(kpx, w)
    pl.set_timing(True, every=3)
    pl.iterate(60)
    ms, launches = pl.read_timing()
    c = pl.counters()
    assert c["full"] and 0 < int(c["iteration"]) < 60, c
    ran = len(range(0, int(c["iteration"]), 3))
    assert launches == [ran] * 4 and all(t > 0 for t in ms), (launches, c["iteration"])
    pl.close()


# the uncapped form (samples_per_node = 0): all active nodes share the buffer
UNCAPPED = {
    "di6": (dict(n_select=900, samples=0, tree_cap=1 << 15), 25),
    "quad12": (dict(n_select=1100, samples=0, tree_cap=1 << 15, grid=(8, 8, 8)), 20),
}


@pytest.mark.parametrize("case", sorted(UNCAPPED))
def test_lockstep_uncapped_form(kpx, ora, case):
    kw, iters = UNCAPPED[case]
    w = W.make_workload(case, 6, **kw)
    P = ora.Problem(w.problem, w.params)
    pl = _planner(kpx, w)
    rep = parity.lockstep(ora, P, pl, iters)
    print(case, rep)
    assert rep["iterations"] == iters and rep["valid"] > 0
    pl.close()


@pytest.mark.parametrize("case,kw", [
    # uncapped: a buffer of 64 slots per region (12^3 regions) keeps every
    # node's share at 64 or more
    ("di6", dict(n_select=64 * 12 ** 3, samples=0, tree_cap=1 << 18, grid=(12, 12, 12))),
    # capped, 64 samples per node
    ("quad12", dict(n_select=300, samples=64, tree_cap=1 << 17, grid=(8, 8, 8))),
])
def test_lockstep_region_minimum_reduced_per_chunk(kpx, ora, case, kw):
    """From 64 samples per node propagate first keeps each chunk's lowest key
    per region (an LDS table) before the region table's atomic minimum: every
    iteration here runs that path, with tree nodes beaten by arrivals, and the
    oracle replays each one."""
    w = W.make_workload(case, 3, **kw)
    P = ora.Problem(w.problem, w.params)
    pl = _planner(kpx, w)
    pl.set_dump(True)
    rep = parity.new_report()
    rep["polished"] = 0
    for _ in range(10):
        pre = pl.snapshot()
        pl.iterate(1)
        parity.check_iteration(ora, P, pl, pre, rep)
        assert int(pl.counters()["samples_per_node"]) >= 64
    print(case, rep)
    assert rep["iterations"] == 10 and rep["valid"] > 0
    st = pl.snapshot()["status"]
    assert int((st == kpx.TERMINAL).sum()) > 0  # nodes were beaten or pruned
    pl.close()


def test_lockstep_long_one_level_scans(kpx, ora):
    """More than 1024 tiles (300,000 slots) and more than 1024 region blocks
    (70^3 = 343,000 regions), summed in one level: each block's offset runs
    over several thousand counts."""
    w = W.make_workload("di6", 6, n_select=300_000, samples=0, tree_cap=1 << 21, grid=(70, 70, 70))
    assert w.params.n_cells > 1024 * 256 and w.params.n_slots > 1024 * 256
    P = ora.Problem(w.problem, w.params)
    pl = _planner(kpx, w)
    rep = parity.lockstep(ora, P, pl, 6)
    print(rep)
    assert rep["iterations"] == 6 and rep["slots"] > 6 * 1024 * 256
    assert pl.counters()["n_tree"] > 100_000
    pl.close()


def test_lockstep_grouped_scans(kpx, ora):
    """More than 8192 tiles (2.2 million slots, 9 groups of 1024) and more than
    8192 region blocks (130^3 = 2,197,000 regions, 9 groups): survivor ranks
    and selection offsets come from the group sums plus the counts within a
    group."""
    w = W.make_workload("di6", 6, n_select=2_200_000, samples=0, tree_cap=1 << 22, grid=(130, 130, 130))
    assert w.params.n_slots > 8192 * 256 and w.params.n_cells > 8192 * 256
    P = ora.Problem(w.problem, w.params)
    pl = _planner(kpx, w)
    rep = parity.lockstep(ora, P, pl, 2)
    print(rep)
    assert rep["iterations"] == 2 and rep["slots"] > 4_000_000
    assert pl.counters()["n_tree"] > 10_000
    pl.close()


@pytest.mark.parametrize("name,iters", [("quad12", 200), ("dubins6", 300)])
def test_full_size_solution_verifies(kpx, ora, name, iters):
    """A full-size plan of the quadrotor and Dubins workloads, re-integrated
    open loop by the oracle in float64 against the exact sets (no margin)."""
    w = W.make_workload(name, 0)
    P = ora.Problem(w.problem, w.params)
    pl = _planner(kpx, w)
    pl.iterate(iters)
    sol = pl.solution()
    print(name, "first solution at iteration", pl.counters()["first_solution_iteration"],
          "cost", sol["cost"] if sol["found"] else None)
    assert sol["found"], pl.counters()
    rep = ora.verify(P, sol["controls"], sol["steps"], sol["states"], float(sol["cost_field"])
                     if w.problem.cost == "TIME" else float(sol["cost"]))
    assert rep["ok"], rep
    pl.close()
