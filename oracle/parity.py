"""Helpers that compare the HIP planner with the float64 oracle (test infrastructure).

Lockstep: the oracle starts from the GPU's pre-iteration snapshot (float32
values widened), replays the same iteration with the same Philox samples, and
adopts the GPU's decision only where its own decision lies within the flag
band of a threshold (and the GPU's is one of the outcomes that band allows).
After that, every integer result must agree exactly.
"""

from __future__ import annotations

import numpy as np

EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)
STATE_RTOL = 1e-4   # states within 1e-4 * max(1, |x_oracle|)
PATH_RTOL = 1e-5    # path-length costs: float32 sums against float64
# polished controls: lr times a float32 against a float64 gradient (relative
# error ~1e-5 after up to 64 RK4 steps), i.e. ~1e-7 of the control per step
POLISH_UTOL = 1e-5


def key_cost(key, cost_kind):
    hi = (np.asarray(key, dtype=np.uint64) >> np.uint64(32)).astype(np.uint32)
    if cost_kind == "TIME":
        return hi.astype(np.float64)
    return hi.view(np.float32).astype(np.float64)


def field_to_cost(field, cost_kind):
    f = np.asarray(field, dtype=np.uint32)
    return f.astype(np.float64) if cost_kind == "TIME" else f.view(np.float32).astype(np.float64)


def oracle_tree_from_snapshot(O, P, snap, cells_cap=None):
    """An oracle Tree holding exactly the GPU's tree (float32 widened)."""
    c = snap["counters"]
    n = int(c["n_tree"])
    tr = O.Tree(P, cells_cap=cells_cap)
    kind = P.problem.cost
    tr.x[:n, : P.d] = snap["state"].T.astype(np.float64)
    tr.u[:n, : P.m] = snap["control"].T
    tr.steps[:n] = snap["steps"]
    tr.parent[:n] = snap["parent"]
    tr.cost[:n] = field_to_cost(snap["cost"], kind)
    tr.cell[:n] = snap["cell"]
    tr.status[:n] = snap["status"]
    tr.icount[:n] = snap["icount"]
    tbl = snap["cell_table"]
    reached = np.flatnonzero(tbl != EMPTY)
    tr.tbl_id[:] = -1
    tr.tbl_cost[:] = np.inf
    tr.tbl_id[reached] = (tbl[reached] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    tr.tbl_cost[reached] = key_cost(tbl[reached], kind)
    sol = np.uint64(c["solution_key"])
    tr.set_scalars(n_tree=n, cursor=int(c["cursor"]), iter=int(c["iteration"]),
                   first_sol_iter=int(c["first_solution_iteration"]), full=int(c["full"]))
    if sol != EMPTY:
        tr.set_scalars(sol_cost=float(key_cost(sol, kind)), sol_id=int(sol & np.uint64(0xFFFFFFFF)))
    else:
        tr.set_scalars(sol_cost=np.inf, sol_id=-1)
    return tr


def hints_from_dump(dump):
    return {
        "first_invalid": dump["first_invalid"].astype(np.int32),
        "cell": dump["cell"].astype(np.int64),
        "goal": dump["goal"].astype(np.uint8),
        "survivor": dump["survivor"].astype(np.uint8),
    }


def compare_candidates(P, tr, dump, report):
    """Slot by slot: the oracle's candidates (after hint adoption) against the GPU dump."""
    c = tr.cands.view()
    S = tr.cands.n_slots
    assert dump["n_slots"] == S, (dump["n_slots"], S)
    if S == 0:
        return
    kind = P.problem.cost
    np.testing.assert_array_equal(dump["parent"], c["parent"])
    np.testing.assert_array_equal(dump["steps"], c["n"])
    # the float32 controls are the same numbers on both sides (one fmaf each)
    np.testing.assert_array_equal(dump["control"].T, c["u"][:, : P.m])
    np.testing.assert_array_equal(dump["first_invalid"], c["first_invalid"])
    valid = c["valid"].astype(bool)
    np.testing.assert_array_equal(dump["cell"][valid], c["cell"][valid])
    np.testing.assert_array_equal(dump["goal"][valid], c["goal"][valid])
    np.testing.assert_array_equal(dump["survivor"], c["survivor"])
    xs_g = dump["state"].T[valid].astype(np.float64)
    xs_o = c["xn"][valid, : P.d]
    err = np.abs(xs_g - xs_o) / np.maximum(1.0, np.abs(xs_o))
    assert err.size == 0 or err.max() <= STATE_RTOL, err.max()
    gk = dump["key"][valid]
    ids = (gk & np.uint64(0xFFFFFFFF)).astype(np.int64)
    np.testing.assert_array_equal(ids, tr_n_tree_before(report) + np.flatnonzero(valid))
    gc = key_cost(gk, kind)
    oc = c["cost"][valid]
    if kind == "TIME":
        np.testing.assert_array_equal(gc, oc)
    else:
        assert np.all(np.abs(gc - oc) <= PATH_RTOL * np.maximum(1.0, oc))
    report["slots"] += S
    report["valid"] += int(valid.sum())
    report["flagged"] += int((c["flags"] != 0).sum())
    report["max_state_err"] = max(report["max_state_err"], float(err.max()) if err.size else 0.0)


def tr_n_tree_before(report):
    return report["n_tree_before"]


def compare_trees(P, tr, snap, report, polished=None):
    """The oracle's post-iteration tree against the GPU's.  `polished` marks
    nodes whose control both sides polished (float32 against float64
    gradient steps): their controls agree to POLISH_UTOL, the rest exactly."""
    kind = P.problem.cost
    c = snap["counters"]
    n = int(c["n_tree"])
    assert tr.n_tree == n, (tr.n_tree, n)
    np.testing.assert_array_equal(snap["parent"], tr.parent[:n])
    np.testing.assert_array_equal(snap["cell"], tr.cell[:n])
    np.testing.assert_array_equal(snap["status"], tr.status[:n])
    np.testing.assert_array_equal(snap["icount"].astype(np.int32), tr.icount[:n])
    np.testing.assert_array_equal(snap["steps"], tr.steps[:n])
    gu, ou = snap["control"].T, tr.u[:n, : P.m]
    loose = np.zeros(n, bool) if polished is None else polished[:n]
    np.testing.assert_array_equal(gu[~loose], ou[~loose])
    if loose.any():
        du = np.abs(gu[loose].astype(np.float64) - ou[loose]) / np.maximum(1.0, np.abs(ou[loose]))
        assert du.max() <= POLISH_UTOL, du.max()
    gcost = field_to_cost(snap["cost"], kind)
    if kind == "TIME":
        np.testing.assert_array_equal(gcost, tr.cost[:n])
    else:
        assert np.all(np.abs(gcost - tr.cost[:n]) <= PATH_RTOL * np.maximum(1.0, tr.cost[:n]))
    xs = snap["state"].T.astype(np.float64)
    err = np.abs(xs - tr.x[:n, : P.d]) / np.maximum(1.0, np.abs(tr.x[:n, : P.d]))
    assert err.max() <= STATE_RTOL
    tbl = snap["cell_table"]
    assert int(tr.c.n_cells) == len(tbl), (int(tr.c.n_cells), len(tbl))
    reached = tbl != EMPTY
    tid, tco = tr.tbl_id[: len(tbl)], tr.tbl_cost[: len(tbl)]
    np.testing.assert_array_equal(reached, tid >= 0)
    np.testing.assert_array_equal((tbl[reached] & np.uint64(0xFFFFFFFF)).astype(np.int64), tid[reached])
    kc = key_cost(tbl[reached], kind)
    if kind == "TIME":
        np.testing.assert_array_equal(kc, tco[reached])
    else:
        assert np.all(np.abs(kc - tco[reached]) <= PATH_RTOL * np.maximum(1.0, kc))
    sol = np.uint64(c["solution_key"])
    if sol == EMPTY:
        assert tr.c.sol_id == -1
    else:
        assert int(sol & np.uint64(0xFFFFFFFF)) == tr.c.sol_id
    assert int(c["first_solution_iteration"]) == tr.c.first_sol_iter
    assert int(c["cursor"]) == tr.c.cursor
    assert int(c["iteration"]) == tr.c.iter
    assert int(c["n_select"]) == tr.c.last_n_sel
    assert int(c["samples_per_node"]) == tr.cands.k
    assert int(c["n_valid"]) == tr.c.last_n_valid
    assert int(c["n_survivors"]) == tr.c.last_n_surv
    assert int(c["substeps"]) == tr.cands.substeps_total


def new_report():
    return {"iterations": 0, "slots": 0, "valid": 0, "flagged": 0, "max_state_err": 0.0,
            "n_tree_before": 0}


def polished_nodes(pre, post, dump):
    """The GPU's edge-polish decisions of this iteration: a mask over the
    post-iteration tree of the nodes whose polished edge it accepted, and the
    per-inserted-node hints (first invalid step, end region, goal bit of the
    polished edge) that the oracle may adopt where its own decision of that
    same test is flagged within band."""
    n0, n1 = int(pre["counters"]["n_tree"]), int(post["counters"]["n_tree"])
    acc = dump["polish_accepted"].astype(bool)
    assert acc.size == n1 - n0, (acc.size, n1 - n0)
    mask = np.zeros(n1, bool)
    mask[n0:n1] = acc
    hints = {"polish_first_invalid": dump["polish_first_invalid"].astype(np.int32),
             "polish_cell": dump["polish_cell"].astype(np.int64),
             "polish_goal": dump["polish_goal"].astype(np.uint8),
             "polish_accepted": dump["polish_accepted"].astype(np.uint8)}
    return mask, hints


def check_iteration(O, P, planner, pre, report):
    """The planner has just run one iteration from the snapshot `pre` (with
    its expansions recorded): the oracle replays that iteration from `pre`
    and every decision is compared."""
    dump = planner.read_dump()
    post = planner.snapshot()
    tr = oracle_tree_from_snapshot(O, P, pre)
    report["n_tree_before"] = tr.n_tree
    mask, polish_hints = polished_nodes(pre, post, dump)
    hints = hints_from_dump(dump)
    hints.update(polish_hints)
    rc = tr.step(hints)
    assert rc == O.OK
    compare_candidates(P, tr, dump, report)
    if P.c.polish_steps > 0:
        # the accept decision of every polished edge, exactly
        n_ins = int(post["counters"]["n_tree"]) - report["n_tree_before"]
        np.testing.assert_array_equal(dump["polish_accepted"], tr.cands.polished[:n_ins])
    compare_trees(P, tr, post, report, polished=mask)
    report["polished"] += int(mask.sum())
    report["iterations"] += 1


def lockstep(O, P, planner, iterations, report=None):
    """Runs `iterations` GPU iterations, replaying each one in the oracle."""
    report = report or new_report()
    report.setdefault("polished", 0)
    planner.set_dump(True)
    for _ in range(iterations):
        pre = planner.snapshot()
        if pre["counters"]["full"]:
            break
        planner.iterate(1)
        check_iteration(O, P, planner, pre, report)
    return report


def lockstep_batch(O, Ps, planners, batch, iterations):
    """Runs `iterations` batched iterations of planners (made with recording
    on before the batch was), replaying every query's iteration in the oracle.
    A query whose tree is full must stay exactly as it was."""
    reports = [dict(new_report(), polished=0, full_at=None) for _ in planners]
    for _ in range(iterations):
        pres = [p.snapshot() for p in planners]
        batch.iterate(1)
        for q, (P, p, pre, rep) in enumerate(zip(Ps, planners, pres, reports)):
            if pre["counters"]["full"]:
                post = p.snapshot()
                assert post["counters"] == pre["counters"], q
                for k in ("parent", "status", "cell_table"):
                    np.testing.assert_array_equal(post[k], pre[k], err_msg=f"query {q}: {k}")
                continue
            check_iteration(O, P, p, pre, rep)
            if p.counters()["full"] and rep["full_at"] is None:
                rep["full_at"] = rep["iterations"]
    return reports
