"""GPU checks at the benchmark workloads' full sizes, in the launch
configuration the benchmark times: sampled slots replayed one by one in the
oracle, plus tree invariants that hold at any size."""

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


def check_tree_invariants(kpx, snap, n_slots_max, n_cells):
    n = int(snap["counters"]["n_tree"])
    par = snap["parent"].astype(np.int64)
    assert par[0] == -1 and np.all(par[1:] >= 0) and np.all(par[1:] < np.arange(1, n))
    st = snap["status"]
    live = np.flatnonzero(st != kpx.TERMINAL)
    cells = snap["cell"][live]
    assert len(np.unique(cells)) == len(cells)  # one live node per region
    tbl = snap["cell_table"]
    assert np.all((tbl[cells] & np.uint64(0xFFFFFFFF)).astype(np.int64) == live)
    owners = (tbl[tbl != parity.EMPTY] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    assert np.all(st[owners] != kpx.TERMINAL) and len(owners) == len(live)
    # the owner's cost field is the region's cost
    assert np.all((tbl[tbl != parity.EMPTY] >> np.uint64(32)).astype(np.uint32) ==
                  snap["cost"][owners])


@pytest.mark.parametrize("name,warm", [("quad12", 12), ("dubins6", 12), ("di6", 40),
                                       ("quad12_paper", 6), ("dubins6_paper", 6), ("di6_paper", 10),
                                       ("quad12_paper_small", 2)])
def test_full_size_sampled_slots(kpx, ora, name, warm):
    sampled_slots_check(kpx, ora, W.make_workload(name, 0), warm)


def test_sampled_slots_root_with_nine_million_samples(kpx, ora):
    """The uncapped form's first iterations give one node 9 million samples:
    a chunk's parent bound (255 parents times the samples per node) no longer
    fits 32 bits.  The root's expansion and the next iteration's."""
    w = W.make_workload("quad12", 0, n_select=9_000_000, samples=0, tree_cap=1 << 24)
    sampled_slots_check(kpx, ora, w, 0)
    sampled_slots_check(kpx, ora, w, 1)


def sampled_slots_check(kpx, ora, w, warm):
    name = w.name
    P = ora.Problem(w.problem, w.params)
    pl = kpx.Planner(w.problem, w.params)
    pl.iterate(warm)
    pre = pl.snapshot()
    pl.set_dump(True)
    pl.iterate(1)
    dump = pl.read_dump()
    post = pl.snapshot()
    S = dump["n_slots"]
    c1 = post["counters"]
    assert S > 0 and S == int(c1["n_select"]) * int(c1["samples_per_node"]) <= w.params.n_slots
    it = int(pre["counters"]["iteration"])
    n0 = int(pre["counters"]["n_tree"])
    rng = np.random.default_rng(0)
    slots = rng.choice(S, size=min(S, 400), replace=False)
    kind = w.problem.cost
    flagged = 0
    for s in slots:
        u, n = ora.sample(P, it, int(s))
        assert n == dump["steps"][s]
        np.testing.assert_array_equal(u[: P.m], dump["control"][:, s])
        par = int(dump["parent"][s])
        x0 = pre["state"][:, par].astype(np.float64)
        e = ora.propagate_edge(P, x0, u, n, int(dump["first_invalid"][s]))
        flagged += e["flags"] != 0
        assert e["first_invalid"] == dump["first_invalid"][s]
        if e["first_invalid"]:
            continue
        xg = dump["state"][:, s].astype(np.float64)
        assert np.all(np.abs(xg - e["xn"]) <= parity.STATE_RTOL * np.maximum(1, np.abs(e["xn"])))
        cell, _ = ora.cell_of(P, e["xn"], hint=int(dump["cell"][s]))
        assert cell == dump["cell"][s]
        key = np.uint64(dump["key"][s])
        assert int(key & np.uint64(0xFFFFFFFF)) == n0 + int(s)
        pc = parity.field_to_cost(pre["cost"][par:par + 1], kind)[0]
        ec = n if kind == "TIME" else e["length"]
        kc = parity.key_cost(np.array([key]), kind)[0]
        if kind == "TIME":
            assert kc == pc + ec
        else:
            assert abs(kc - (pc + ec)) <= parity.PATH_RTOL * max(1.0, kc)
    print(name, "slots", S, "checked", len(slots), "flagged", flagged)
    check_tree_invariants(kpx, post, S, w.params.n_cells)
    # survivors: each is its region's owner now, appended in slot order
    surv = np.flatnonzero(dump["survivor"][:S])
    n1 = int(post["counters"]["n_tree"])
    assert n1 - n0 == len(surv)
    tbl = post["cell_table"]
    np.testing.assert_array_equal((tbl[dump["cell"][surv]] & np.uint64(0xFFFFFFFF)).astype(np.int64),
                                  n0 + np.arange(len(surv)))
    pl.close()


@pytest.mark.parametrize("name,warm", [("quad12", None), ("dubins6", 40), ("dubins6_paper", 12)])
def test_full_size_lockstep_at_the_benchmark_shapes(kpx, ora, name, warm):
    """Three iterations at a workload's own size, replayed slot by slot by the
    oracle.  quad12: once its selection is full (4096 x 32 slots: 512 per
    propagate chunk, two per lane, sorted by length and refilled from the
    queue).  dubins6: after 40 iterations; its capped selection never exceeds
    the ~2,000 regions with an active owner (of 16,384), so its lanes hold one
    slot each.  dubins6_paper, the uncapped form with a 300,000-slot buffer:
    more than 1,024 slots per block, so one chunk of up to 2,048 (about 1,170
    here) and two to three slots per lane of 512-thread blocks, the Dubins
    sort and refill path."""
    w = W.make_workload(name, 0)
    P = ora.Problem(w.problem, w.params)
    pl = kpx.Planner(w.problem, w.params)
    if warm is None:
        for _ in range(100):
            pl.iterate(1)
            if int(pl.counters()["n_select"]) == w.params.n_select:
                break
        pl.iterate(1)  # the next selection is full as well (the region count only grows)
        assert int(pl.counters()["n_select"]) == w.params.n_select
    else:
        pl.iterate(warm)
    rep = parity.lockstep(ora, P, pl, 3)
    print(name, rep)
    assert rep["iterations"] == 3
    if warm is None:
        assert rep["slots"] == 3 * w.params.n_slots, rep
    if name == "dubins6_paper":
        assert rep["slots"] > 3 * 1024 * 256, rep  # more than 1,024 slots per block on 256 CUs
    pl.close()
