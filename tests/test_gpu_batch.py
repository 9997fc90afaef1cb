"""Batched queries through the C ABI: each query of a batch computes exactly
what it computes alone, with plain launches and with replayed HIP graphs, and
the oracle replays every iteration of a batch of queries at their own sizes."""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("state", "control", "steps", "parent", "cost", "cell", "status", "icount", "cell_table")


@pytest.fixture(scope="module")
def kpx():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_02846_amd as K

    K.lib()
    return K


def _small_batch(n, seed, n_select_max=300):
    ws = W.batch_workloads(seed, n)
    for w in ws:  # test-sized: fewer nodes per iteration, same scenes and capacities
        w.params.n_select = min(w.params.n_select, n_select_max)
    return ws


def _same(a, b, what):
    for k in KEYS:
        np.testing.assert_array_equal(a[k], b[k], err_msg=f"{what}: {k}")
    assert a["counters"] == b["counters"], what


def test_batch_matches_each_query_alone(kpx):
    ws = _small_batch(10, 3)
    alone = []
    for w in ws:
        p = kpx.Planner(w.problem, w.params)
        p.iterate(25)
        p.sync()
        alone.append(p.snapshot())
        p.close()
    ps = [kpx.Planner(w.problem, w.params) for w in ws]
    b = kpx.Batch(ps)
    b.iterate(25)
    states = b.sync()
    for q, (p, a) in enumerate(zip(ps, alone)):
        _same(p.snapshot(), a, f"query {q}")
    # the capacities include trees that fill up within the run
    assert kpx.FULL in states and kpx.OK in states, states
    b.close()
    for p in ps:
        p.close()


def test_batch_with_many_region_blocks_matches_alone(kpx):
    """A query of 70^3 regions (more than 1024 region blocks) and one of more
    than 1024 tiles, batched with a small one, graph-replayed: each tree is
    the one the query grows alone."""
    ws = [W.make_workload("di6", 6, n_select=2000, samples=0, tree_cap=1 << 20, grid=(70, 70, 70)),
          W.make_workload("di6", 7, n_select=300_000, samples=0, tree_cap=1 << 20),
          W.make_workload("quad12", 2, n_select=64, samples=8, tree_cap=1 << 16, grid=(8, 8, 8))]
    alone = []
    for w in ws:
        p = kpx.Planner(w.problem, w.params)
        p.iterate(8)
        alone.append(p.snapshot())
        p.close()
    ps = [kpx.Planner(w.problem, w.params) for w in ws]
    b = kpx.Batch(ps, graph=True)
    b.iterate(8)
    b.sync()
    for q, (p, a) in enumerate(zip(ps, alone)):
        _same(p.snapshot(), a, f"query {q}")
    b.close()
    for p in ps:
        p.close()


def test_batch_graph_replays_match_plain_launches(kpx):
    ws = _small_batch(8, 5, n_select_max=200)
    plain = [kpx.Planner(w.problem, w.params) for w in ws]
    graph = [kpx.Planner(w.problem, w.params) for w in ws]
    bp, bg = kpx.Batch(plain), kpx.Batch(graph, graph=True)
    for step in (6, 5, 4, 1, 6):  # replays of two iterations, and odd remainders
        bp.iterate(step)
        bg.iterate(step)
        for q, (a, g) in enumerate(zip(plain, graph)):
            _same(a.snapshot(), g.snapshot(), f"query {q} after {step}")
        plain[0].counters()  # eager work between replays
    for b in (bp, bg):
        b.close()
    for p in plain + graph:
        p.close()


def test_batch_rejects_bad_groupings(kpx):
    ws = _small_batch(3, 7)
    ps = [kpx.Planner(w.problem, w.params) for w in ws]
    with pytest.raises(kpx.KPXError):
        kpx.Batch([ps[0], ps[0]])  # the same handle twice
    ps[1].set_dump(True)
    b = kpx.Batch(ps)  # a recording handle keeps recording in the batch
    b.iterate(1)
    ps[1].set_dump(False)  # ... but may not switch it off while batched
    with pytest.raises(kpx.KPXError):
        b.iterate(1)
    b.close()
    ps[2].iterate(1)  # out of step with the others
    with pytest.raises(kpx.KPXError):
        kpx.Batch(ps)
    for p in ps:
        p.close()


def test_autotuner_scores_every_candidate(kpx):
    """The samples-per-node autotuner runs each candidate on a sample of each
    model's queries and keeps the one with the lowest median time to a first
    solution; with_samples keeps N*K and fits an iteration in half the tree."""
    from paper_2602_02846_amd.autotune import autotune_samples, with_samples

    ws = _small_batch(8, 3)
    chosen, scores = autotune_samples(ws, candidates=(4, 8), iterations=12, sample=3)
    assert set(chosen) == {w.problem.dynamics for w in ws}
    for model, k in chosen.items():
        assert set(scores[model]) == {4, 8}
        assert all(v > 0 for v in scores[model].values())
        assert scores[model][k] == min(scores[model].values())
    for w in ws:
        w2 = with_samples(w, 8)
        assert w2.params.samples_per_node == 8
        assert w2.params.n_select * 8 <= max(8, w.params.n_select * w.params.samples_per_node)
        assert w2.params.n_select * 8 <= w.params.tree_cap // 2 or w2.params.n_select == 1
        assert w.params.samples_per_node != 8 or w2.params.n_select == w.params.n_select


def test_batch_threads_per_block_keep_the_trees(kpx):
    """Two waves per SIMD for one model's propagate (and back) leave every
    tree as each query grows it alone; graphs are captured again."""
    ws = _small_batch(6, 9)
    alone = []
    for w in ws:
        p = kpx.Planner(w.problem, w.params)
        p.iterate(16)
        alone.append(p.snapshot())
        p.close()
    ps = [kpx.Planner(w.problem, w.params) for w in ws]
    b = kpx.Batch(ps, graph=True)
    b.set_threads("DI6", 512)
    b.iterate(6)
    b.set_threads("QUAD12", 512)
    b.iterate(6)
    b.set_threads("DI6", 256)
    b.iterate(4)
    b.sync()
    for q, (p, a) in enumerate(zip(ps, alone)):
        _same(p.snapshot(), a, f"query {q}")
    with pytest.raises(kpx.KPXError):
        b.set_threads("DI6", 384)
    b.close()
    for p in ps:
        p.close()


def test_autotuner_tries_threads_per_block(kpx):
    from paper_2602_02846_amd.autotune import autotune

    ws = _small_batch(6, 4)
    chosen, scores = autotune(ws, candidates=(8,), threads=(256, 512), iterations=10, sample=2)
    for model, (k, nt) in chosen.items():
        assert set(scores[model]) == {(8, 256), (8, 512)}
        assert scores[model][(k, nt)] == min(scores[model].values())


def test_batch_of_uncapped_queries_matches_each_alone(kpx):
    """Queries in the uncapped form (every active node, lambda per iteration
    from the device state) batched with capped ones."""
    ws = _small_batch(6, 11)
    for w in ws[::2]:
        w.params.samples_per_node = 0
        w.params.n_select = 600
    alone = []
    for w in ws:
        p = kpx.Planner(w.problem, w.params)
        p.iterate(15)
        p.sync()
        alone.append(p.snapshot())
        p.close()
    ps = [kpx.Planner(w.problem, w.params) for w in ws]
    b = kpx.Batch(ps, graph=True)
    b.iterate(15)
    b.sync()
    for q, (p, a) in enumerate(zip(ps, alone)):
        _same(p.snapshot(), a, f"query {q}")
    b.close()
    for p in ps:
        p.close()


def test_batch_lockstep_with_the_oracle(kpx, ora):
    """Seven queries of the batched workload at their own sizes (double
    integrators and quadrotors with 94 to 250 boxes, capacities 2^13 to 2^18,
    one of which fills up in the tenth iteration), graph-replayed as one
    batch: every query's every iteration is replayed by the oracle."""
    from oracle import parity

    ws = W.batch_workloads(0, 40)
    pick = [2, 3, 4, 14, 19, 21, 33]
    chosen = [ws[q] for q in pick]
    assert {w.problem.dynamics for w in chosen} == {"DI6", "QUAD12"}
    assert all(w.problem.n_boxes >= 94 for w in chosen)
    Ps = [ora.Problem(w.problem, w.params) for w in chosen]
    ps = [kpx.Planner(w.problem, w.params) for w in chosen]
    for p in ps:
        p.set_dump(True)
    b = kpx.Batch(ps, graph=True)
    reps = parity.lockstep_batch(ora, Ps, ps, b, 14)
    b.close()
    for q, (w, rep) in zip(pick, zip(chosen, reps)):
        print(q, w.problem.dynamics, w.problem.n_boxes, rep)
        assert rep["iterations"] >= 10 and rep["valid"] > 0, (q, rep)
    # the query that fills up does so mid-run, and stays as it was afterwards
    assert reps[0]["full_at"] is not None and reps[0]["iterations"] < 14, reps[0]
    for p in ps:
        p.close()


def test_batch_of_four_model_cost_groups_matches_each_alone(kpx):
    """Four (model, cost) groups, each iterating on a stream of its own:
    double integrators (time), quadrotors (time and path length) and Dubins
    airplanes (path length), graph-replayed in odd runs with eager work
    between them; every query's tree is the one it grows alone."""
    from workloads.scenes import small_overrides

    ws = []
    for seed in range(2):
        ws.append(W.make_workload("di6", seed, **small_overrides("di6")))
        ws.append(W.make_workload("quad12", seed, **small_overrides("quad12")))
        ws.append(W.make_workload("quad12", seed + 2, cost="PATH_LENGTH", **small_overrides("quad12")))
        ws.append(W.make_workload("dubins6", seed, **small_overrides("dubins6")))
    assert len({(w.problem.dynamics, w.problem.cost) for w in ws}) == 4
    alone = []
    for w in ws:
        p = kpx.Planner(w.problem, w.params)
        p.iterate(17)
        alone.append(p.snapshot())
        p.close()
    ps = [kpx.Planner(w.problem, w.params) for w in ws]
    b = kpx.Batch(ps, graph=True)
    for step in (5, 4, 1, 7):
        b.iterate(step)
        ps[0].counters()  # eager work between the runs
    b.sync()
    for q, (p, a) in enumerate(zip(ps, alone)):
        _same(p.snapshot(), a, f"query {q}")
    b.close()
    for p in ps:
        p.close()
