"""Benchmark: propagated edges/s of the Kino-PAX+ iteration on one MI355X.

A step is one planner iteration (select -> propagate -> prune -> insert) of one
query on the 12D quadrotor workload (4096 nodes x 32 samples per iteration,
64-box wall with two slots, 16^3 x 2^3 regions, tree capacity 2^21).  Inputs
live in HBM before timing starts; every count stays on the device.

Prints one JSON line.  `roofline` covers the dominant kernel (propagate, bound
by float32 ALU work); `cpu_baseline` is the float64 oracle replaying the same
workload on the host from the GPU tree at the start of the timed region.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic float32 FLOPs of one RK4 substep (FMA = 2, each transcendental,
# reciprocal or square root = 1): 13 per integrated component for the stage
# and combination updates plus four evaluations of f.
#   DI6      6 components, f has no arithmetic                  -> 78
#   QUAD12  12 components, f = 6 sin/cos + 1 rcp + 35 mul/FMA   -> 156 + 4 * 42 = 324
#   DUBINS6  6 components, f = 4 sin/cos + 4 mul                 -> 78 + 4 * 8 = 110
# The path-length cost integrates one more component and its rate
# (speed: 3 FMA-equivalents + sqrt for DI6/QUAD12, none for DUBINS6).
FLOPS_PER_SUBSTEP = {
    ("DI6", "TIME"): 78, ("DI6", "PATH_LENGTH"): 78 + 13 + 4 * 6,
    ("QUAD12", "TIME"): 324, ("QUAD12", "PATH_LENGTH"): 324 + 13 + 4 * 6,
    ("DUBINS6", "TIME"): 110, ("DUBINS6", "PATH_LENGTH"): 110 + 13,
}
PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32 (256 CUs x 2.4 GHz x 256 FLOP/clk)
PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = ("paper_2602_02846_amd/csrc/kpx.hip", "paper_2602_02846_amd/csrc/kpx_device.hpp")


def measured_traffic(workload):
    """HBM bytes per propagate launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, calibrated against a plain copy), or
    None when there is none or the kernel sources changed since it was taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"propagate_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    fields = {}
    with open(path) as fh:
        for line in fh:
            k, sep, v = line.partition(":")
            if sep:
                fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256") != h.hexdigest():
        return None
    try:
        return int(fields["propagate_hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=150)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="quad12",
                    choices=["di6", "quad12", "dubins6", "di6_paper", "quad12_paper", "dubins6_paper",
                             "batch256"])
    ap.add_argument("--queries", type=int, default=256, help="queries of the batch256 workload")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batch256: skip the sequential per-query comparison")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="bound on the oracle CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--solution-seeds", type=int, default=10,
                    help="queries (seeds) for the median time to first solution and cost")
    ap.add_argument("--solution-iters", type=int, default=200,
                    help="iteration budget of each of those queries")
    ap.add_argument("--no-timing", action="store_true", help="no per-kernel HIP events")
    ap.add_argument("--time-all", action="store_true",
                    help="HIP events around all four kernels (default: propagate only)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="first run one device-to-device copy of this size (counter calibration)")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {a.gpus} is not supported "
              "(the planner query runs on a single device)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2602_02846_amd as K
    import workloads as W

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if a.workload == "batch256":
        return bench_batch(a)
    K.lib()  # fails loudly when the HIP library is missing
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if a.copy_bytes > 0:
        src = torch.ones(a.copy_bytes, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = W.make_workload(a.workload, a.seed)
    prob, prm = w.problem, w.params

    planner = K.Planner(prob, prm, device="cuda:0")
    print(f"[bench] {a.workload}: {prm.n_select} x {prm.samples_per_node} slots, "
          f"{prm.n_cells} regions, cap {prm.tree_cap}; warmup {a.warmup}", file=sys.stderr,
          flush=True)
    planner.iterate(a.warmup)
    planner.sync()
    snap_start = planner.snapshot() if not a.no_cpu_baseline else None
    c0 = planner.counters()
    if not a.no_timing:
        # HIP events around propagate (the roofline kernel), or all four kernels
        planner.set_timing(15 if a.time_all else 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    planner.iterate(a.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rc = planner.sync()
    c1 = planner.counters()
    done = int(c1["iteration"] - c0["iteration"])
    st = planner.stats(int(c0["iteration"]), done) if done > 0 else None
    edges = int((st["n_select"].astype(np.int64) * st["samples_per_node"]).sum()) if done else 0
    substeps = int(st["substeps"].sum()) if done else 0
    elapsed = t1 - t0
    value = edges / elapsed if elapsed > 0 else 0.0
    print(f"[bench] timed {done} iterations in {elapsed * 1e3:.2f} ms, {edges} edges, "
          f"status {rc}", file=sys.stderr, flush=True)

    roofline = None
    kernel_ms = None
    if not a.no_timing:
        ms, launches = planner.read_timing()
        kernel_ms = {name: (ms[i] / launches[i] if launches[i] else None)
                     for i, name in enumerate(["propagate", "prune_flags", "insert",
                                               "finalize_select"]) if launches[i]}
        if launches[0]:
            fl = FLOPS_PER_SUBSTEP[(prob.dynamics, prob.cost)] * substeps / launches[0]
            avg_s = ms[0] / launches[0] / 1e3
            achieved = fl / avg_s / 1e12
            roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                        "traffic": measured_traffic(a.workload)}

    # time to first solution and cost, from device timestamps of this query
    it_done = int(c1["iteration"])
    all_st = planner.stats(max(0, it_done - 65536), min(it_done, 65536))
    rate = planner.clock_rate_khz() * 1e3
    first_it = int(c1["first_solution_iteration"])
    sol = planner.solution()
    t_first = None
    if first_it >= 0 and all_st.size and all_st["iteration"][0] == 0:
        t_first = float((int(all_st["t_end"][first_it]) - int(all_st["t_begin"][0])) / rate * 1e3)

    planner.close()
    sols = solution_medians(K, W, a) if a.solution_seeds > 0 else None

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(w, snap_start, a.cpu_seconds)

    out = {
        "metric": "propagated edges/s", "value": round(value, 1), "unit": "edges/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(elapsed * 1e3 / max(done, 1), 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{a.workload}: {prob.dynamics} {prob.n_boxes} boxes, "
                   + (f"{prm.n_select}x{prm.samples_per_node} expansions/iteration, "
                      if prm.samples_per_node else
                      f"every active node sharing {prm.n_select} expansion slots per iteration, ")
                   + f"{prm.n_cells} regions, cap {prm.tree_cap}",
                   "seed": a.seed, "iterations_timed": done, "edges_timed": edges,
                   "substeps_timed": substeps, "cost": prob.cost},
        "roofline": roofline,
        "kernel_ms": kernel_ms,
        "time_to_first_solution_ms": t_first,
        "first_solution_iteration": first_it,
        "solution_cost": sol["cost"] if sol["found"] else None,
        "solutions": sols,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def solution_medians(K, W, a):
    """Median device-timed time to first solution and median solution cost of
    the plain planner over seeds 0 .. solution_seeds - 1 of the workload, each
    run for solution_iters iterations (or until its tree is full)."""
    from paper_2602_02846_amd.autotune import first_solution_ms

    times, costs = [], []
    for seed in range(a.solution_seeds):
        w = W.make_workload(a.workload, seed)
        p = K.Planner(w.problem, w.params)
        p.iterate(a.solution_iters)
        p.sync()
        t = first_solution_ms(p, a.solution_iters)
        if t is not None:
            times.append(t)
            costs.append(p.solution()["cost"])
        p.close()
    return {"queries": a.solution_seeds, "iterations": a.solution_iters, "solved": len(times),
            "time_to_first_solution_ms_median": round(float(np.median(times)), 3) if times else None,
            "cost_median": round(float(np.median(costs)), 4) if costs else None,
            "cost_unit": "s" if W.make_workload(a.workload, 0).problem.cost == "TIME" else "length"}


def bench_batch(a):
    """Independent queries (half double integrators, half quadrotors, seeded
    scenes of 4..256 boxes, capacities 2^10..2^18) iterated as one batch of
    graph-replayed launches, against the same queries run one after another."""
    import torch

    import paper_2602_02846_amd as K
    import workloads as W
    from paper_2602_02846_amd.autotune import autotune_samples, first_solution_ms, with_samples

    K.lib()
    torch.cuda.set_device(0)
    ws = W.batch_workloads(a.seed, a.queries)
    chosen, scores = autotune_samples(ws)
    ws = [with_samples(w, chosen[w.problem.dynamics]) for w in ws]
    print(f"[bench] batch of {len(ws)} queries; samples per node {chosen} "
          f"(autotuner medians, ms: {scores})", file=sys.stderr, flush=True)
    n_iter = a.warmup + a.steps

    planners = [K.Planner(w.problem, w.params) for w in ws]
    batch = K.Batch(planners, graph=True)
    torch.cuda.synchronize()
    tb0 = time.perf_counter()
    batch.iterate(a.warmup)
    batch.sync()
    c0 = [p.counters() for p in planners]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.iterate(a.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    batch.sync()
    elapsed, whole = t1 - t0, t1 - tb0
    edges = substeps = 0
    flops = 0.0
    for p, w, c in zip(planners, ws, c0):
        c1 = p.counters()
        done = int(c1["iteration"] - c["iteration"])
        if done > 0:
            st = p.stats(int(c["iteration"]), done)
            e = int((st["n_select"].astype(np.int64) * st["samples_per_node"]).sum())
            sub = int(st["substeps"].sum())
            edges += e
            substeps += sub
            flops += FLOPS_PER_SUBSTEP[(w.problem.dynamics, w.problem.cost)] * sub
    t_first = [first_solution_ms(p, n_iter) for p in planners]
    solved = [t for t in t_first if t is not None]
    costs = [p.solution()["cost"] for p in planners if p.counters()["first_solution_iteration"] >= 0]
    batch.close()
    for p in planners:
        p.close()
    print(f"[bench] batch: {a.steps} iterations in {elapsed * 1e3:.1f} ms, {edges} edges", file=sys.stderr,
          flush=True)

    seq = None
    if not a.no_sequential:
        t_seq, seq_edges_timed = 0.0, 0
        for w in ws:
            p = K.Planner(w.problem, w.params)
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            p.iterate(n_iter)
            p.sync()
            torch.cuda.synchronize()
            t_seq += time.perf_counter() - s0
            p.close()
        seq = {"whole_run_s": round(t_seq, 4), "queries_per_s": round(len(ws) / t_seq, 2)}

    achieved = flops / elapsed / 1e12 if elapsed > 0 else 0.0
    out = {
        "metric": "propagated edges/s", "value": round(edges / elapsed, 1), "unit": "edges/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(elapsed * 1e3 / max(a.steps, 1), 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch{len(ws)}: {len(ws) // 2} DI6 + {len(ws) - len(ws) // 2} QUAD12 "
                               "queries, 4..256 boxes, caps 2^10..2^18, graph-replayed batch",
                   "seed": a.seed, "samples_per_node": chosen, "edges_timed": edges,
                   "substeps_timed": substeps},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None,
                     "scope": "RK4 FLOPs over whole iterations (all kernels)"},
        "queries_per_s": round(len(ws) / whole, 2),
        "batch_whole_run_s": round(whole, 4),
        "sequential": seq,
        "speedup_vs_sequential": round(seq["whole_run_s"] / whole, 2) if seq else None,
        "solved": len(solved), "queries": len(ws),
        "time_to_first_solution_ms_median": round(float(np.median(solved)), 3) if solved else None,
        "solution_cost_median": round(float(np.median(costs)), 4) if costs else None,
    }
    print(json.dumps(out))


def cpu_baseline(w, snap, seconds):
    """The float64 oracle (single thread, as written) stepping the same tree."""
    from oracle import oracle as O
    from oracle import parity

    P = O.Problem(w.problem, w.params)
    tr = parity.oracle_tree_from_snapshot(O, P, snap)
    edges = 0
    iters = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        rc = tr.step()
        if rc != O.OK:
            break
        edges += tr.cands.n_slots
        iters += 1
    el = time.perf_counter() - t0
    return {"value": round(edges / el, 1) if el > 0 else None, "unit": "edges/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{iters} iterations of the same query from the GPU tree at the start of "
                      f"the timed region ({edges} expansions, {el:.1f} s, float64, one thread)"}


if __name__ == "__main__":
    main()
