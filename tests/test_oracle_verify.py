"""Pins of the trajectory verifier: it accepts a planned solution and rejects
each kind of defect (collision, bound violation, missed goal, wrong cost,
wrong start)."""

import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def solved(ora):
    w = W.make_workload("di6", 2)
    P = ora.Problem(w.problem, w.params)
    tr = ora.run(P, 80)
    assert tr.c.sol_id >= 0
    ctrl, steps, states = tr.path_to(tr.c.sol_id)
    return P, w, tr, ctrl, steps, states


def test_accepts_the_planned_solution(ora, solved):
    P, w, tr, ctrl, steps, states = solved
    rep = ora.verify(P, ctrl, steps, states, tr.c.sol_cost)
    assert rep["ok"] and rep["cost"] == steps.sum() == tr.c.sol_cost
    assert rep["min_clearance"] > 0


def test_rejects_wrong_cost(ora, solved):
    P, w, tr, ctrl, steps, states = solved
    assert not ora.verify(P, ctrl, steps, states, tr.c.sol_cost + 1)["ok"]


def test_rejects_missing_last_edge(ora, solved):
    P, w, tr, ctrl, steps, states = solved
    rep = ora.verify(P, ctrl[:-1], steps[:-1], states[:-1], float(steps[:-1].sum()))
    assert not rep["reaches_goal"] and not rep["ok"]


def test_rejects_wrong_start(ora, solved):
    P, w, tr, ctrl, steps, states = solved
    bad = states.copy()
    bad[0, 0] += 1e-3
    assert not ora.verify(P, ctrl, steps, bad, tr.c.sol_cost)["starts_at_init"]


def test_rejects_collision(ora, solved):
    P, w, tr, ctrl, steps, states = solved
    # a scene with a box over the goal region swallows the trajectory's end
    w2 = W.make_workload("di6", 2)
    c = w2.problem.goal_center
    w2.problem.boxes = np.concatenate([w2.problem.boxes, [[*(c - 0.2), *(c + 0.2)]]]).astype(np.float32)
    P2 = ora.Problem(w2.problem, w2.params)
    rep = ora.verify(P2, ctrl, steps, states, tr.c.sol_cost)
    assert not rep["collision_free"] and not rep["ok"] and rep["first_bad_edge"] >= 0


def test_rejects_bound_violation(ora, solved):
    P, w, tr, ctrl, steps, states = solved
    big = ctrl.copy()
    big[:] = 1.0  # full acceleration on every edge exceeds |v| <= 1
    rep = ora.verify(P, big, steps * 0 + 30, None, 0.0)
    assert not rep["within_bounds"] or not rep["collision_free"]


def test_empty_plan_only_from_inside_the_goal(ora):
    """No edge: accepted exactly when the start lies in the goal ball."""
    w = W.make_workload("di6", 2)
    P = ora.Problem(w.problem, w.params)
    none_u, none_n = np.zeros((0, 4), np.float32), np.zeros(0, np.int32)
    rep = ora.verify(P, none_u, none_n, w.problem.x_init[:6].reshape(1, 6), 0.0)
    assert not rep["ok"] and not rep["reaches_goal"]
    w.problem.x_init = w.problem.x_init.copy()
    w.problem.x_init[:3] = np.asarray(w.problem.goal_center, np.float32)
    P = ora.Problem(w.problem, w.params)
    rep = ora.verify(P, none_u, none_n, w.problem.x_init[:6].reshape(1, 6), 0.0)
    assert rep["ok"] and rep["reaches_goal"] and rep["cost"] == 0.0
