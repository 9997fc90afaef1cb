"""Edge polish of inserted nodes (kpx_set_polish) through the C ABI against
the float64 oracle: lockstep iterations in which both sides polish every
inserted quadrotor node (the oracle adopting the GPU's accept decision only
where its own is within the flag band), argument checks, and re-verification
of a polished plan by the oracle."""

import numpy as np
import pytest

import workloads as W

from oracle import parity

pytestmark = pytest.mark.gpu

LOCK = dict(n_select=260, samples=9, tree_cap=1 << 16, grid=(8, 8, 8))
POLISH = dict(steps=3, lr=0.01)


@pytest.fixture(scope="module")
def kpx():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_02846_amd as K

    K.lib()
    return K


@pytest.mark.parametrize("seed", [5, 6])
def test_lockstep_with_polish(kpx, ora, seed):
    w = W.make_workload("quad12", seed, **LOCK)
    P = ora.Problem(w.problem, w.params, polish=POLISH)
    pl = kpx.Planner(w.problem, w.params)
    pl.set_polish(**POLISH)
    rep = parity.lockstep(ora, P, pl, 20)
    print(seed, rep)
    assert rep["iterations"] == 20
    assert rep["polished"] > 0
    pl.close()


POLISH_PATH = dict(steps=3, lr=0.01, w_len=1.0)


@pytest.mark.parametrize("seed", [5, 8])
def test_lockstep_with_path_length_polish(kpx, ora, seed):
    """The path-length cost: a polished edge that is shorter lowers its node's
    cost and its region's key (and the solution's, for a goal node); the
    oracle replays every decision, adopting the GPU's only within the band."""
    w = W.make_workload("quad12", seed, cost="PATH_LENGTH", **LOCK)
    P = ora.Problem(w.problem, w.params, polish=POLISH_PATH)
    pl = kpx.Planner(w.problem, w.params)
    pl.set_polish(**POLISH_PATH)
    lowered = 0
    rep = parity.new_report()
    for _ in range(20):
        pre = pl.snapshot()
        n0 = int(pre["counters"]["n_tree"])
        rep = parity.lockstep(ora, P, pl, 1, rep)
        post = pl.snapshot()
        # nodes whose polished edge was accepted: their cost is below the
        # unpolished arrival's key, which the dump still holds
        dump = pl.read_dump()
        surv = np.flatnonzero(dump["survivor"][: dump["n_slots"]])
        keys = (dump["key"][surv] >> np.uint64(32)).astype(np.uint32).view(np.float32)
        costs = post["cost"][n0:n0 + len(surv)].view(np.float32)
        acc = dump["polish_accepted"][: len(surv)].astype(bool)
        assert np.all(costs[acc] < keys[acc]) and np.all(costs[~acc] == keys[~acc])
        lowered += int(acc.sum())
    print(seed, rep, "lowered", lowered)
    assert rep["iterations"] == 20
    assert lowered > 0
    pl.close()


def test_lockstep_with_goal_only_path_length_polish(kpx, ora):
    """Only the nodes inserted in the goal set are polished (the others stay
    as inserted); a shorter polished edge lowers the solution key.  The goal
    ball is moved to the start's side of the wall (0.3, 0.5, 0.5), radius 0.1,
    so that this small query inserts goal nodes early."""
    pol = dict(POLISH_PATH, steps=6, goal_only=True)
    w = W.make_workload("quad12", 0, cost="PATH_LENGTH", **LOCK)
    w.problem.goal_center = np.array([0.3, 0.5, 0.5], np.float32)
    w.problem.goal_radius = float(np.float32(0.1))
    P = ora.Problem(w.problem, w.params, polish=pol)
    pl = kpx.Planner(w.problem, w.params)
    pl.set_polish(**pol)
    rep = parity.new_report()
    goal_nodes = 0
    for _ in range(40):
        rep = parity.lockstep(ora, P, pl, 1, rep)
        d = pl.read_dump()
        S = d["n_slots"]
        goal_nodes += int((d["goal"][:S].astype(bool) & d["survivor"][:S].astype(bool)).sum())
    c = pl.counters()
    print(rep, "goal nodes inserted", goal_nodes, "first solution at", c["first_solution_iteration"])
    assert rep["iterations"] == 40
    assert goal_nodes > 0 and c["first_solution_iteration"] >= 0
    pl.close()


def test_polish_arguments(kpx):
    di = W.make_workload("di6", 0)
    pd = kpx.Planner(di.problem, di.params)
    with pytest.raises(kpx.KPXError):
        pd.set_polish(3)
    pd.set_polish(0)  # off is always accepted
    pd.close()
    qp = W.make_workload("quad12", 0, cost="PATH_LENGTH", **LOCK)
    pp = kpx.Planner(qp.problem, qp.params)
    pp.set_polish(3, w_len=1.0)  # the path-length cost is polished too
    pp.set_polish(3, w_len=1.0, goal_only=True)
    with pytest.raises(kpx.KPXError):
        pp.set_polish(3, w_len=float("nan"))
    pp.close()
    q = W.make_workload("quad12", 0, **LOCK)
    pq = kpx.Planner(q.problem, q.params)
    for bad in (dict(steps=17), dict(steps=-1), dict(steps=3, lr=-1.0), dict(steps=3, lr=float("nan")),
                dict(steps=3, w_goal=float("inf"))):
        with pytest.raises(kpx.KPXError):
            pq.set_polish(**bad)
    pq.set_polish(**POLISH)
    with pytest.raises(kpx.KPXError):
        kpx.Batch([pq])
    pq.set_polish(0)
    b = kpx.Batch([pq])
    b.close()
    pq.close()


def test_polish_off_is_the_plain_planner(kpx):
    w = W.make_workload("quad12", 7, **LOCK)
    a = kpx.Planner(w.problem, w.params)
    b = kpx.Planner(w.problem, w.params)
    b.set_polish(**POLISH)
    b.set_polish(0)
    a.iterate(10)
    b.iterate(10)
    sa, sb = a.snapshot(), b.snapshot()
    for k in ("state", "control", "parent", "cell", "status"):
        np.testing.assert_array_equal(sa[k], sb[k])
    a.close()
    b.close()


def test_polished_plan_reverifies(kpx, ora):
    w = W.make_workload("quad12", 1)  # full size: 4096 nodes x 32 samples
    P = ora.Problem(w.problem, w.params)
    pl = kpx.Planner(w.problem, w.params)
    pl.set_polish(**POLISH)
    pl.iterate(200)
    c = pl.counters()
    print("polished run:", c["n_tree"], "nodes, first solution at iteration", c["first_solution_iteration"])
    sol = pl.solution()
    if not sol["found"]:
        pytest.skip("no solution within 200 iterations for this seed")
    rep = ora.verify(P, sol["controls"], sol["steps"], sol["states"], float(sol["cost_field"]))
    assert rep["ok"], rep
    pl.close()


def test_lockstep_polish_with_uncapped_form_and_refinement(kpx, ora):
    """Polish in the uncapped form (lambda from the device state), across a
    refinement of the regions."""
    import dataclasses

    w = W.make_workload("quad12", 9, n_select=1100, samples=0, tree_cap=1 << 15, grid=(4, 4, 4))
    w.params.refine_max = 2
    P = ora.Problem(w.problem, w.params, polish=POLISH)
    P2 = ora.Problem(w.problem, dataclasses.replace(w.params, grid=(8, 8, 8)), polish=POLISH)
    pl = kpx.Planner(w.problem, w.params)
    pl.set_polish(**POLISH)
    rep = parity.lockstep(ora, P, pl, 8)
    pre = pl.snapshot()
    pl.refine(2)
    post = pl.snapshot()
    tr = parity.oracle_tree_from_snapshot(ora, P, pre, cells_cap=P2.n_cells)
    assert tr.refine(P2, 2, hint_cell=post["cell"]) == ora.OK
    np.testing.assert_array_equal(post["cell"], tr.cell[: len(post["cell"])])
    rep2 = parity.lockstep(ora, P2, pl, 8)
    print(rep, rep2)
    assert rep["iterations"] == 8 and rep2["iterations"] == 8
    assert rep["polished"] + rep2["polished"] > 0
    pl.close()
