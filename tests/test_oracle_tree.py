"""Pins of the oracle's node-set logic: Alg. 3 on hand-built trees with
hand-computed outcomes, the rotating selection, and invariants that every
iteration of a full run must keep (brute-force region minimum, additive cost,
one live node per region, monotone region and solution costs)."""

import numpy as np
import pytest

import workloads as W

A, I, T = 0, 1, 2  # ACTIVE, INACTIVE, TERMINAL


def _tree(ora, nodes, i_max=2, n_select=2, **kw):
    """nodes: list of (parent, cell, cost, status, icount); region owners are
    the lowest (cost, id) per cell unless overridden by the caller."""
    w = W.make_workload("di6", 0, i_max=i_max, n_select=n_select, samples=2, tree_cap=64, **kw)
    P = ora.Problem(w.problem, w.params)
    tr = ora.Tree(P, cap=64)
    for i, (par, cell, cost, st, ic) in enumerate(nodes):
        tr.parent[i], tr.cell[i], tr.cost[i], tr.status[i], tr.icount[i] = par, cell, cost, st, ic
        if cost < tr.tbl_cost[cell] or (cost == tr.tbl_cost[cell] and i < tr.tbl_id[cell]):
            tr.tbl_cost[cell], tr.tbl_id[cell] = cost, i
    tr.set_scalars(n_tree=len(nodes))
    return tr


def test_prune_all_best_stays_active(ora):
    tr = _tree(ora, [(-1, 0, 0, A, 0), (0, 1, 5, A, 0), (1, 2, 9, A, 0), (0, 3, 6, A, 0)])
    tr.prune()
    assert tr.status[:4].tolist() == [A, A, A, A]


def test_prune_beaten_node_terminal_and_descendants_inactive(ora):
    # node 5 beats node 1 in cell 1; 2, 3 (children of 1) and 4 (grandchild) go dormant
    nodes = [(-1, 0, 0, A, 0), (0, 1, 5, A, 0), (1, 2, 9, A, 0), (1, 3, 8, A, 0),
             (2, 4, 12, A, 0), (0, 1, 4, A, 0), (0, 6, 7, A, 0)]
    tr = _tree(ora, nodes)
    assert tr.tbl_id[1] == 5
    tr.prune()
    assert tr.status[:7].tolist() == [A, T, I, I, I, A, A]
    assert tr.icount[:7].tolist() == [0] * 7


def test_prune_inactive_counts_then_wakes(ora):
    # node 2 is dormant and region-best; I_max = 2: counts 1 -> 2 (dormant), 3 (> I_max: wakes)
    nodes = [(-1, 0, 0, A, 0), (0, 1, 5, T, 0), (1, 2, 9, I, 1), (0, 1, 4, A, 0)]
    tr = _tree(ora, nodes)
    tr.prune()
    assert tr.status[2] == I and tr.icount[2] == 2
    tr.prune()
    assert tr.status[2] == A and tr.icount[2] == 3
    # woken and still best: left alone although its parent stays beaten (Alg. 3)
    tr.prune()
    assert tr.status[2] == A and tr.icount[2] == 3


def test_prune_dormant_or_woken_but_beaten_is_terminal(ora):
    nodes = [(-1, 0, 0, A, 0), (0, 1, 5, I, 1), (0, 2, 5, A, 3), (0, 1, 3, A, 0), (0, 2, 4, A, 0)]
    tr = _tree(ora, nodes)
    tr.prune()
    assert tr.status[:5].tolist() == [A, T, T, A, A]
    assert tr.icount[1] == 1  # a beaten dormant node does not count


def test_prune_grandparent_beaten(ora):
    # 3's parent 2 is best, grandparent 1 is beaten by 4
    nodes = [(-1, 0, 0, A, 0), (0, 1, 6, A, 0), (1, 2, 9, A, 0), (2, 3, 14, A, 0), (0, 1, 5, A, 0)]
    tr = _tree(ora, nodes)
    tr.prune()
    assert tr.status[:5].tolist() == [A, T, I, I, A]


def test_prune_ties_go_to_the_lower_id(ora):
    nodes = [(-1, 0, 0, A, 0), (0, 1, 5, A, 0), (0, 1, 5, A, 0)]
    tr = _tree(ora, nodes)
    tr.prune()
    assert tr.status[:3].tolist() == [A, A, T]


def test_select_rotates_from_the_cursor(ora):
    nodes = [(-1, 10, 0, A, 0), (0, 3, 5, A, 0), (0, 7, 5, A, 0), (0, 20, 5, A, 0),
             (0, 12, 5, I, 0), (0, 15, 5, T, 0)]
    tr = _tree(ora, nodes, n_select=2)
    tr.set_scalars(cursor=8)
    sel, cur = tr.select()
    assert sel.tolist() == [0, 3] and cur == 21
    tr.set_scalars(cursor=21)
    sel, cur = tr.select()
    assert sel.tolist() == [1, 2] and cur == 8
    tr.set_scalars(cursor=0)
    sel, cur = tr.select()
    assert sel.tolist() == [1, 2]


def test_select_takes_all_when_few_are_active(ora):
    nodes = [(-1, 10, 0, I, 0), (0, 3, 5, A, 0)]
    tr = _tree(ora, nodes, n_select=4)
    sel, cur = tr.select()
    assert sel.tolist() == [1] and cur == 4


def _run_with_invariants(ora, w, iterations, polish=None, on_step=None):
    P = ora.Problem(w.problem, w.params, polish=polish)
    tr = ora.Tree(P)
    assert tr.init() == ora.OK
    nc = P.n_cells
    K = w.params.samples_per_node
    prev_tbl = tr.tbl_cost.copy()
    prev_sol = np.inf
    sols = []
    for it in range(iterations):
        n0 = tr.n_tree
        pre_status = tr.status[:n0].copy()
        pre_cost = tr.cost[:n0].copy()
        pre_cell = tr.cell[:n0].copy()
        pre_owner = tr.tbl_id.copy()
        sel, _ = tr.select()
        rc = tr.step()
        if rc == ora.FULL:
            break
        c = tr.cands.view()
        S = tr.cands.n_slots
        if K == 0:
            # uncapped form: every active node up to the buffer, sharing it evenly
            n_active = int(np.count_nonzero(pre_status == A))
            assert len(sel) == min(n_active, w.params.n_select)
            k_it = max(1, w.params.n_select // len(sel)) if len(sel) else 1
            assert tr.cands.k == k_it and S == len(sel) * k_it <= w.params.n_select
        else:
            k_it = K
            assert tr.cands.k == K
        assert S == len(sel) * k_it
        assert np.array_equal(c["parent"], np.repeat(sel, k_it))
        # selected nodes were ACTIVE
        assert np.all(pre_status[sel] == A)
        # brute-force region minimum over incumbents and this iteration's arrivals
        best = {}
        for cell in set(c["cell"][c["valid"] == 1].tolist()):
            if pre_owner[cell] >= 0:
                best[cell] = (pre_cost[pre_owner[cell]], pre_owner[cell])
        for s in range(S):
            if c["valid"][s]:
                key = (c["cost"][s], n0 + s)
                cell = int(c["cell"][s])
                if cell not in best or key < best[cell]:
                    best[cell] = key
        winners = {v[1] - n0 for v in best.values() if v[1] >= n0}
        surv = set(np.flatnonzero(c["survivor"]).tolist())
        assert surv == winners
        # survivors appended in slot order
        order = sorted(surv)
        assert [int(c["new_index"][s]) for s in order] == list(range(n0, n0 + len(order)))
        n1 = tr.n_tree
        assert n1 == n0 + len(order) <= n0 + min(nc, S)
        # additive cost, parent before child, exact re-integration of stored edges
        for i in range(n0, n1):
            p = tr.parent[i]
            assert 0 <= p < i
            ec = tr.steps[i] if w.problem.cost == "TIME" else None
            z = ora.integrate(P, tr.x[p, : P.d], tr.u[i, : P.m].astype(float), int(tr.steps[i]))
            assert np.array_equal(z[: P.d], tr.x[i, : P.d])
            # the stored edge is valid in the planning set (substep by substep)
            assert ora.propagate_edge(P, tr.x[p, : P.d], tr.u[i, : P.m], int(tr.steps[i]))["first_invalid"] == 0
            if ec is not None:
                assert tr.cost[i] == tr.cost[p] + ec
            else:
                assert abs(tr.cost[i] - (tr.cost[p] + z[P.d])) <= 1e-12 * max(1.0, tr.cost[i])
            assert tr.cell[i] == ora.cell_of(P, tr.x[i, : P.d])[0]
        # one live node per region, and it is the region's owner
        live = np.flatnonzero(tr.status[:n1] != T)
        cells = tr.cell[live]
        assert len(set(cells.tolist())) == len(cells)
        assert np.all(tr.tbl_id[cells] == live)
        reached = tr.tbl_id >= 0
        owners = tr.tbl_id[reached]
        assert np.all(tr.status[owners] != T)
        assert np.all(tr.tbl_cost[reached] == tr.cost[owners])
        # region costs and the solution never increase
        assert np.all(tr.tbl_cost <= prev_tbl)
        prev_tbl = tr.tbl_cost.copy()
        assert tr.c.sol_cost <= prev_sol
        prev_sol = tr.c.sol_cost
        if tr.c.sol_id >= 0:
            sols.append(int(tr.c.sol_id))
            assert ora.goal_test(P, tr.x[tr.c.sol_id, : P.d])[0]
        if on_step:
            on_step(tr, c, n0, n1)
    return P, tr, sols


@pytest.mark.parametrize("cost", ["TIME", "PATH_LENGTH"])
def test_full_run_invariants_double_integrator(ora, cost):
    w = W.make_workload("di6", 1, iterations=80, cost=cost)
    P, tr, sols = _run_with_invariants(ora, w, 80)
    assert tr.n_tree > 1000
    assert sols, "no solution in 80 iterations"
    # the returned trajectory re-verifies
    ctrl, steps, states = tr.path_to(tr.c.sol_id)
    rep = ora.verify(P, ctrl, steps, states, tr.c.sol_cost)
    assert rep["ok"], rep
    assert rep["max_gap"] < 1e-6  # stored states are passed as float32


def test_full_run_invariants_quadrotor_small(ora):
    w = W.make_workload("quad12", 2, n_select=48, samples=6, grid=(8, 8, 8), tree_cap=1 << 15)
    _run_with_invariants(ora, w, 40)


def test_polish_keeps_the_invariants_and_lowers_the_loss(ora):
    """Edge polish of inserted quadrotor nodes: every invariant above still
    holds (stored edges re-integrate exactly to the stored states, regions and
    costs unchanged by construction), some nodes are polished, and each
    polished control has a lower tied loss than the sampled one."""
    import copy

    w = W.make_workload("quad12", 2, n_select=48, samples=6, grid=(8, 8, 8), tree_cap=1 << 15)
    grown = copy.deepcopy(w.problem)
    b = np.asarray(w.problem.boxes, np.float32).reshape(-1, 6)
    m = np.float32(w.problem.margin)
    grown.boxes = np.concatenate([b[:, :3] - m, b[:, 3:] + m], axis=1).astype(np.float32)
    D = ora.DiffProblem(grown, w.params.dt)
    seen = {"new": 0, "polished": 0}

    def check(tr, c, n0, n1):
        for s in np.flatnonzero(c["survivor"]):
            i = int(c["new_index"][s])
            seen["new"] += 1
            u0 = c["u"][s, :4].astype(np.float64)
            u1 = tr.u[i, :4].astype(np.float64)
            if np.array_equal(u0, u1):
                continue
            seen["polished"] += 1
            x0 = tr.x[tr.parent[i]]
            n = int(tr.steps[i])
            assert ora.diff_loss(D, x0, np.tile(u1, 4), n) < ora.diff_loss(D, x0, np.tile(u0, 4), n)
            lo, hi = np.asarray(w.problem.u_lo[:4]), np.asarray(w.problem.u_hi[:4])
            assert np.all(u1 >= lo) and np.all(u1 <= hi)

    _run_with_invariants(ora, w, 25, polish=dict(steps=3, lr=0.01), on_step=check)
    assert seen["polished"] > seen["new"] // 4, seen


def test_polish_tied_gradient_is_the_sum_over_segments(ora):
    b = W.diff_workload(5, n_edges=3)
    D = ora.DiffProblem(b.problem, b.dt)
    for e in range(3):
        u = np.tile(b.u[e, :4].astype(np.float64), 4)
        g16 = ora.diff_grad(D, b.x0[e], u, int(b.n[e]))
        g4 = ora.diff_grad_tied(D, b.x0[e], u, int(b.n[e]))
        np.testing.assert_allclose(g4, g16.reshape(4, 4).sum(0), rtol=1e-12, atol=1e-12)


def test_full_run_invariants_uncapped_form(ora):
    """samples_per_node = 0: every active node (up to a 600-slot buffer) with
    lambda = max(1, floor(600 / |selected|)) samples, checked against the
    active nodes counted before each step."""
    w = W.make_workload("di6", 4, n_select=600, samples=0, tree_cap=1 << 15)
    P, tr, sols = _run_with_invariants(ora, w, 30)
    assert tr.n_tree > 300


def test_full_run_invariants_dubins_small(ora):
    w = W.make_workload("dubins6", 3, n_select=48, samples=6, grid=(16, 16, 8), tree_cap=1 << 15)
    _run_with_invariants(ora, w, 40)


def test_coarse_grid_double_integrator_cannot_leave_the_start_region(ora):
    """With 8^3 regions an edge from rest moves at most 0.045 (< 0.075 to the
    face) and every arrival in the start region costs more than the root."""
    w = W.make_workload("di6", 0, grid=(8, 8, 8))
    P = ora.Problem(w.problem, w.params)
    tr = ora.Tree(P)
    tr.init()
    for _ in range(20):
        tr.step()
    assert tr.n_tree == 1


def test_capacity_precheck_stops_cleanly(ora):
    w = W.make_workload("di6", 0, n_select=16, samples=4, tree_cap=1 + 64 + 30)
    P = ora.Problem(w.problem, w.params)
    tr = ora.Tree(P)
    assert tr.init() == ora.OK
    rcs = [tr.step() for _ in range(50)]
    assert ora.FULL in rcs
    k = rcs.index(ora.FULL)
    n = tr.n_tree
    assert n + 64 > tr.c.cap
    assert all(rc == ora.FULL for rc in rcs[k:])
    assert tr.n_tree == n


def test_init_rejects_bad_problems(ora):
    w = W.make_workload("di6", 0)
    w.problem.x_init[:3] = w.problem.boxes[0, :3] + 1e-3  # inside a box
    P = ora.Problem(w.problem, w.params)
    assert ora.Tree(P).init() == ora.ERR_INVALID_START
    w = W.make_workload("di6", 0)
    w.params.steps_min = 0
    assert ora.Tree(ora.Problem(w.problem, w.params)).init() == ora.ERR_ARG
    w = W.make_workload("dubins6", 0)
    w.params.vel_sign_bins = 1
    assert ora.Tree(ora.Problem(w.problem, w.params)).init() == ora.ERR_ARG


def _coarse(cell, grid_new, f, vel):
    bits = cell % 8 if vel else 0
    s = cell // 8 if vel else cell
    gz, gy = grid_new[2], grid_new[1]
    iz, iy, ix = s % gz, (s // gz) % gy, s // (gz * gy)
    s0 = ((ix // f) * (gy // f) + iy // f) * (gz // f) + iz // f
    return s0 * 8 + bits if vel else s0


@pytest.mark.parametrize("name,kw", [
    ("di6", dict(n_select=100, samples=7, tree_cap=1 << 15, grid=(8, 8, 8))),
    ("quad12", dict(n_select=90, samples=9, tree_cap=1 << 15, grid=(4, 4, 4))),
])
def test_refine_keeps_the_invariants(ora, name, kw):
    """Adaptive decomposition: after 12 iterations the grid is halved per
    axis; every node's region is its state's region in the new grid and lies
    inside its old one, the live nodes own their new regions one each, the
    table holds nothing else, the cursor moved to the first new cell of its
    old one, and 12 more iterations keep one live owner per region."""
    import dataclasses

    w = W.make_workload(name, 3, **kw)
    w.params.refine_max = 2
    vel = bool(w.params.vel_sign_bins)
    P = ora.Problem(w.problem, w.params)
    P2 = ora.Problem(w.problem, dataclasses.replace(w.params, grid=tuple(2 * g for g in w.params.grid)))
    tr = ora.Tree(P, cells_cap=P2.n_cells)
    assert tr.init() == ora.OK
    for _ in range(12):
        assert tr.step() == ora.OK
    n = tr.n_tree
    old_cell = tr.cell[:n].copy()
    old_status = tr.status[:n].copy()
    old_cursor = int(tr.c.cursor)
    assert tr.refine(P2, 2) == ora.OK
    assert int(tr.c.n_cells) == P2.n_cells == 8 * P.n_cells
    for i in range(n):
        c = int(tr.cell[i])
        assert c == ora.cell_of(P2, tr.x[i, : P.d])[0]
        assert _coarse(c, P2.params.grid, 2, vel) == old_cell[i]
    np.testing.assert_array_equal(tr.status[:n], old_status)
    live = np.flatnonzero(tr.status[:n] != T)
    assert len(set(tr.cell[live].tolist())) == len(live)
    np.testing.assert_array_equal(tr.tbl_id[tr.cell[live]], live)
    np.testing.assert_array_equal(tr.tbl_cost[tr.cell[live]], tr.cost[live])
    assert int((tr.tbl_id[: P2.n_cells] >= 0).sum()) == len(live)
    assert _coarse(int(tr.c.cursor), P2.params.grid, 2, vel) == old_cursor
    for _ in range(12):
        rc = tr.step()
        if rc == ora.FULL:
            break
        m = tr.n_tree
        live = np.flatnonzero(tr.status[:m] != T)
        assert len(set(tr.cell[live].tolist())) == len(live)
        np.testing.assert_array_equal(tr.tbl_id[tr.cell[live]], live)
        for i in range(n, m):
            assert tr.cell[i] == ora.cell_of(P2, tr.x[i, : P.d])[0]
    assert tr.n_tree > n


def test_polish_closed_form_without_scene_terms(ora):
    """With the obstacle and goal terms off the tied loss is n dt + 4 w_ctrl |u|^2,
    so each projected step scales the control by 1 - 8 lr w_ctrl (the box
    contains the scaled control: thrust >= 0, torques symmetric); every
    polished node's control is the sampled one times that factor cubed."""
    w = W.make_workload("quad12", 2, n_select=48, samples=6, grid=(8, 8, 8), tree_cap=1 << 15)
    pol = dict(steps=3, lr=0.01, w_obst=0.0, w_goal=0.0)
    P = ora.Problem(w.problem, w.params, polish=pol)
    f32 = lambda v: float(np.float32(v))  # noqa: E731
    factor = (1.0 - 8.0 * f32(0.01) * f32(0.1)) ** 3
    tr = ora.Tree(P)
    assert tr.init() == ora.OK
    checked = 0
    for _ in range(8):
        assert tr.step() == ora.OK
        c = tr.cands.view()
        for s in np.flatnonzero(c["survivor"]):
            i = int(c["new_index"][s])
            u0 = c["u"][s, :4].astype(np.float64)
            u1 = tr.u[i, :4]
            if np.array_equal(u0.astype(np.float32), u1):
                continue  # rejected: left its region or became invalid
            np.testing.assert_array_equal(u1, (u0 * factor).astype(np.float32))
            checked += 1
    assert checked > 20


def _grown(problem):
    import copy

    g = copy.deepcopy(problem)
    b = np.asarray(problem.boxes, np.float32).reshape(-1, 6)
    m = np.float32(problem.margin)
    g.boxes = np.concatenate([b[:, :3] - m, b[:, 3:] + m], axis=1).astype(np.float32)
    return g


@pytest.mark.parametrize("lr", [0.01, 3.0])
def test_polish_steps_replayed_from_the_tied_gradient(ora, lr):
    """Each polished node's control equals projected steps replayed here from
    the complex-step tied gradient of the loss with the given weights (over the
    grown boxes, towards the goal centre).  lr = 3 overshoots the control box,
    so the projection decides most components."""
    w = W.make_workload("quad12", 4, n_select=48, samples=6, grid=(8, 8, 8), tree_cap=1 << 15)
    pol = dict(steps=2, lr=lr, w_ctrl=0.2, w_obst=0.5, k_obst=40.0, d_safe=0.03, w_goal=2.0)
    P = ora.Problem(w.problem, w.params, polish=pol)
    f = lambda v: float(np.float32(v))  # noqa: E731
    D = ora.DiffProblem(_grown(w.problem), w.params.dt, w_ctrl=0.2, w_obst=0.5, k_obst=40.0, d_safe=0.03,
                        w_goal=2.0)
    lo = np.asarray(w.problem.u_lo[:4], np.float64)
    hi = np.asarray(w.problem.u_hi[:4], np.float64)
    tr = ora.Tree(P)
    assert tr.init() == ora.OK
    checked = clamped = 0
    for _ in range(12):
        assert tr.step() == ora.OK
        c = tr.cands.view()
        for s in np.flatnonzero(c["survivor"]):
            i = int(c["new_index"][s])
            u0 = c["u"][s, :4].astype(np.float64)
            if np.array_equal(u0.astype(np.float32), tr.u[i, :4]):
                continue
            u = u0.copy()
            x0 = tr.x[tr.parent[i]]
            for _ in range(2):
                g = ora.diff_grad_tied(D, x0, np.tile(u, 4), int(tr.steps[i]))
                u = np.clip(u - f(lr) * g, lo, hi)
            clamped += int(np.sum((u == lo) | (u == hi)))
            np.testing.assert_allclose(tr.u[i, :4], u, rtol=1e-6, atol=1e-7)
            checked += 1
    assert checked >= 8
    if lr > 1:
        assert clamped > checked


def test_refinement_that_outgrows_the_capacity_stops_the_tree(ora):
    """Refining grows the survivor bound min(regions, slots); when the tree can
    no longer take one more iteration's bound it is full, and the next step
    reports FULL without changing anything."""
    import dataclasses

    w = W.make_workload("di6", 3, n_select=100, samples=7, tree_cap=1 << 15, grid=(8, 8, 8))
    w.params.refine_max = 2
    P = ora.Problem(w.problem, w.params)
    tr = ora.Tree(P, cells_cap=8 * P.n_cells)
    assert tr.init() == ora.OK
    for _ in range(3):
        assert tr.step() == ora.OK
    n = tr.n_tree
    # a capacity between n + 512 (the bound before) and n + 700 (after: 100 x 7 slots)
    tr.c.cap = n + 600
    P2 = ora.Problem(w.problem, dataclasses.replace(w.params, grid=(16, 16, 16)))
    assert tr.refine(P2, 2) == ora.OK
    assert tr.c.full == 1
    assert tr.step() == ora.FULL
    assert tr.n_tree == n


def test_root_in_the_goal_is_a_solution_of_cost_zero(ora):
    """A start inside the goal set is the empty trajectory of cost 0, found
    before the first iteration, and no later node beats it (every edge costs
    more than 0)."""
    for name in ("di6", "dubins6"):
        w = W.make_workload(name, 1, **dict(W.scenes.small_overrides(name), samples=64))
        w.problem.x_init = w.problem.x_init.copy()
        w.problem.x_init[:3] = np.asarray(w.problem.goal_center, np.float32)
        P = ora.Problem(w.problem, w.params)
        T = ora.Tree(P)
        assert T.init() == ora.OK
        assert (T.c.sol_id, T.c.sol_cost, T.c.first_sol_iter) == (0, 0.0, 0)
        for _ in range(6):
            T.step()
        assert (T.c.sol_id, T.c.sol_cost, T.c.first_sol_iter) == (0, 0.0, 0)
        # (the airplane, heading into the corner, only returns to the start region)
        assert T.n_tree > 1 or name == "dubins6"
        # just outside the planning goal radius there is no such solution
        w.problem.x_init[0] += np.float32(w.problem.goal_radius - w.problem.margin + 1e-3)
        T2 = ora.Tree(ora.Problem(w.problem, w.params))
        if T2.init() == ora.OK:
            assert T2.c.sol_id == -1 and T2.c.first_sol_iter == -1


@pytest.mark.parametrize("name", ["quad12", "dubins6"])
def test_threaded_timing_build_steps_like_the_plain_oracle(ora, name):
    """The OpenMP build that times the oracle on every host core shares the
    expansions among threads; its trees equal the plain build's."""
    w = W.make_workload(name, 1, n_select=64, samples=8, tree_cap=1 << 14)
    P = ora.Problem(w.problem, w.params)
    a, b = ora.Tree(P), ora.Tree(P)
    assert a.init() == ora.OK and b.init() == ora.OK
    for _ in range(12):
        assert a.step() == ora.OK
        assert b.step(threaded=True) == ora.OK
        assert a.cands.substeps_total == b.cands.substeps_total
    n = a.n_tree
    assert n == b.n_tree and n > 100
    for k in ("x", "u", "steps", "parent", "cost", "cell", "status", "icount", "tbl_cost", "tbl_id"):
        np.testing.assert_array_equal(getattr(a, k)[:n] if k not in ("tbl_cost", "tbl_id") else getattr(a, k),
                                      getattr(b, k)[:n] if k not in ("tbl_cost", "tbl_id") else getattr(b, k),
                                      err_msg=k)
    assert ora.lib_threads().ora_threads() >= 1
