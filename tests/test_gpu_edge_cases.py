"""Edge cases of the HIP planner: capacity exhaustion, degenerate sizes, an
unreachable goal, an obstacle-free scene, ragged slot counts."""

import numpy as np
import pytest

import workloads as W

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


def test_tiny_capacity_reports_full_and_stops(kpx, ora):
    w = W.make_workload("di6", 0, n_select=32, samples=4, tree_cap=1 + 128 + 40)
    P = ora.Problem(w.problem, w.params)
    pl = kpx.Planner(w.problem, w.params)
    rcs = []
    for _ in range(60):
        pl.iterate(1)
        rcs.append(pl.sync())
    assert kpx.FULL in rcs
    c = pl.counters()
    assert c["full"] == 1 and c["n_tree"] + 128 > w.params.tree_cap
    assert pl.iterate(5) == kpx.FULL
    assert pl.counters() == c
    # the oracle agrees on when the tree fills
    tr = ora.run(P, 60)
    assert tr.c.full == 1 and tr.n_tree == c["n_tree"] and tr.c.iter == c["iteration"]
    pl.close()


@pytest.mark.parametrize("n_select,k", [(1, 1), (1, 33), (7, 1), (513, 3)])
def test_degenerate_and_ragged_sizes_lockstep(kpx, ora, n_select, k):
    w = W.make_workload("di6", 4, n_select=n_select, samples=k, tree_cap=1 << 15)
    P = ora.Problem(w.problem, w.params)
    pl = kpx.Planner(w.problem, w.params)
    rep = parity.lockstep(ora, P, pl, 12)
    assert rep["iterations"] == 12
    pl.close()


@pytest.mark.parametrize("name", ["di6", "quad12"])
def test_root_in_the_goal_is_a_solution(kpx, ora, name):
    """A start inside the goal set is a solution of cost 0 with no edge, from
    before the first iteration; no inserted node can beat it."""
    w = W.make_workload(name, 2, n_select=64, samples=4, tree_cap=1 << 14)
    w.problem.x_init = w.problem.x_init.copy()
    w.problem.x_init[:3] = np.asarray(w.problem.goal_center, np.float32)
    P = ora.Problem(w.problem, w.params)
    pl = kpx.Planner(w.problem, w.params)
    c = pl.counters()
    assert c["solution_key"] == 0 and c["first_solution_iteration"] == 0
    rep = parity.lockstep(ora, P, pl, 4)
    assert rep["iterations"] == 4
    sol = pl.solution()
    assert sol["found"] and sol["tree_index"] == 0 and sol["n_edges"] == 0 and sol["cost"] == 0.0
    assert sol["first_solution_iteration"] == 0
    rep = ora.verify(P, np.zeros((0, 4), np.float32), np.zeros(0, np.int32), sol["states"], 0.0)
    assert rep["ok"] and rep["reaches_goal"]
    pl.close()


@pytest.mark.parametrize("steps", [(1, 1), (7, 7), (1, 2)])
def test_fixed_and_one_step_durations(kpx, ora, steps):
    """Edges of one RK4 step, and fixed step counts (a single sort bin), in
    lockstep with the oracle; the cost-first form grows the same tree."""
    w = W.make_workload("quad12", 5, n_select=90, samples=9, tree_cap=1 << 15, grid=(8, 8, 8), steps=steps)
    P = ora.Problem(w.problem, w.params)
    pl = kpx.Planner(w.problem, w.params)
    cf = kpx.Planner(w.problem, w.params)
    cf.set_cost_first(True)
    rep = parity.lockstep(ora, P, pl, 10)
    assert rep["iterations"] == 10 and rep["valid"] > 0
    cf.iterate(10)
    a, b = pl.snapshot(), cf.snapshot()
    for k in ("state", "control", "steps", "parent", "cost", "cell", "status", "cell_table"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    assert a["counters"]["n_tree"] > 1
    pl.close()
    cf.close()


def test_unreachable_goal_has_no_solution(kpx):
    w = W.make_workload("di6", 3)
    c = w.problem.goal_center
    w.problem.boxes = np.concatenate(
        [w.problem.boxes, [[c[0] - 0.1, c[1] - 0.1, c[2] - 0.1, 1.0, 1.0, 1.0]]]).astype(np.float32)
    pl = kpx.Planner(w.problem, w.params)
    pl.iterate(120)
    sol = pl.solution()
    assert not sol["found"] and sol["tree_index"] == -1
    assert pl.counters()["first_solution_iteration"] == -1
    pl.close()


def test_no_obstacles_lockstep(kpx, ora):
    w = W.make_workload("quad12", 6, n_select=100, samples=5, grid=(8, 8, 8), tree_cap=1 << 15)
    w.problem.boxes = np.zeros((0, 6), np.float32)
    P = ora.Problem(w.problem, w.params)
    pl = kpx.Planner(w.problem, w.params)
    rep = parity.lockstep(ora, P, pl, 10)
    assert rep["iterations"] == 10
    pl.close()


def test_dump_requires_recording(kpx):
    w = W.make_workload("di6", 0, n_select=8, samples=2)
    pl = kpx.Planner(w.problem, w.params)
    pl.iterate(1)
    with pytest.raises(kpx.KPXError) as e:
        pl.read_dump()
    assert e.value.code == -6
    pl.close()


def test_boxes_on_box_grid_faces_lockstep(kpx, ora):
    """Box faces exactly on the planner's internal box-grid boundaries (multiples
    of 1/16 of the workspace) and many overlapping boxes: the grid lookup must
    agree with the oracle's test against every box."""
    rng = np.random.default_rng(8)
    boxes = []
    while len(boxes) < 120:
        lo = rng.integers(1, 14, size=3) / 16.0
        ext = rng.integers(1, 3, size=3) / 16.0
        b = np.concatenate([lo, lo + ext])
        if np.all(b[:3] <= 0.1) or np.linalg.norm(np.clip([0.95] * 3, b[:3], b[3:]) - 0.95) < 0.08:
            continue
        boxes.append(b)
    w = W.make_workload("di6", 7, n_select=300, samples=9, tree_cap=1 << 16, margin=0.0)
    w.problem.boxes = np.asarray(boxes, np.float32)
    P = ora.Problem(w.problem, w.params)
    pl = kpx.Planner(w.problem, w.params)
    rep = parity.lockstep(ora, P, pl, 25)
    assert rep["iterations"] == 25 and rep["valid"] > 0
    pl.close()
