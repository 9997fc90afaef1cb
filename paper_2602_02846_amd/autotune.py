"""Samples-per-node and threads-per-block autotuner for batches of queries.

For each robot model of a batch, every candidate K (samples per node), with
every candidate propagate block size (256 or 512 threads: one or two waves per
SIMD, the lanes that serve a node's samples), is tried
on a sample of that model's queries, run together as a batch for a fixed
number of iterations; the K whose queries reach a first solution soonest (the
median over the sample of the device-timed span from the first iteration to
the end of the first-solution iteration, unsolved queries counting as the
whole run) is kept.  The node count per iteration is re-clipped for each K so
that one iteration's candidates still fit in half the tree.
"""

from __future__ import annotations

import copy

import numpy as np

from .kpx import Batch, Planner


def first_solution_ms(planner, n_iters: int):
    """Device-timed span from the first iteration's start to the end of the
    first-solution iteration, or None if unsolved."""
    c = planner.counters()
    it = int(c["first_solution_iteration"])
    if it < 0:
        return None
    n = min(int(c["iteration"]), n_iters)
    st = planner.stats(int(c["iteration"]) - n, n)
    if st.size == 0 or st["iteration"][0] != 0 or it >= st.size:
        return None
    rate = planner.clock_rate_khz() * 1e3
    return float((int(st["t_end"][it]) - int(st["t_begin"][0])) / rate * 1e3)


def with_samples(w, k: int):
    """A copy of workload w with k samples per node (node count re-clipped)."""
    w2 = copy.deepcopy(w)
    w2.params.samples_per_node = int(k)
    w2.params.n_select = max(1, min(int(w.params.n_select) * int(w.params.samples_per_node) // int(k),
                                    (int(w.params.tree_cap) // 2) // int(k)))
    return w2


def autotune_samples(workloads, candidates=(8, 16, 32), iterations: int = 40, sample: int = 16):
    """Returns {model: K} for the models present in `workloads`, and the
    per-candidate scores {model: {K: median ms}} (256 threads per block)."""
    chosen, scores = autotune(workloads, candidates, (256,), iterations, sample)
    return ({m: kt[0] for m, kt in chosen.items()},
            {m: {kt[0]: v for kt, v in sc.items()} for m, sc in scores.items()})


def autotune(workloads, candidates=(8, 16, 32), threads=(256, 512), iterations: int = 40,
             sample: int = 16):
    """Returns {model: (K, threads)} for the models present in `workloads`,
    and the per-candidate scores {model: {(K, threads): median ms}}."""
    chosen, scores = {}, {}
    for model in sorted({w.problem.dynamics for w in workloads}):
        ws = [w for w in workloads if w.problem.dynamics == model][:sample]
        scores[model] = {}
        for k, nt in [(k, nt) for k in candidates for nt in threads]:
            planners = [Planner(p.problem, p.params) for p in (with_samples(w, k) for w in ws)]
            batch = Batch(planners, graph=False)
            batch.set_threads(model, nt)
            batch.iterate(iterations)
            batch.sync()
            ts = []
            for p in planners:
                t = first_solution_ms(p, iterations)
                ts.append(t if t is not None else float("inf"))
            # unsolved queries count as the whole run: the span of the longest solved one, doubled
            finite = [t for t in ts if np.isfinite(t)]
            cap = 2.0 * max(finite) if finite else 1e9
            scores[model][(k, nt)] = float(np.median([min(t, cap) for t in ts]))
            batch.close()
            for p in planners:
                p.close()
        chosen[model] = min(scores[model], key=scores[model].get)
    return chosen, scores
