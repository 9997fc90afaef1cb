"""Pins of the float64 oracle of the differentiable edge rollout: its states
against the (pinned) planner oracle's RK4, its signed distance against brute
force, its loss recomposed from its states, its complex-step gradient against
central differences and a closed form."""

import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def setup(ora):
    b = W.diff_workload(0, n_edges=64)
    D = ora.DiffProblem(b.problem, b.dt)
    return ora, b, D


def test_segments(setup):
    ora, _, _ = setup
    assert [ora.diff_segment(k, 20) for k in range(20)] == [0] * 5 + [1] * 5 + [2] * 5 + [3] * 5
    # n = 22: boundaries floor(j n / 4) = 0, 5, 11, 16
    assert [ora.diff_segment(k, 22) for k in range(22)] == [0] * 5 + [1] * 6 + [2] * 5 + [3] * 6


def test_states_follow_the_planner_rk4(setup):
    ora, b, D = setup
    w = W.make_workload("quad12", 0)
    P = ora.Problem(w.problem, w.params)
    for e in range(4):
        n = int(b.n[e])
        _, st = ora.diff_loss(D, b.x0[e], b.u[e], n, states=True)
        x = b.x0[e].astype(np.float64)
        k = 0
        for j in range(4):
            steps = (j + 1) * n // 4 - j * n // 4
            x = ora.integrate(P, x, b.u[e, 4 * j:4 * j + 4].astype(np.float64), steps)[:12]
            k += steps
            np.testing.assert_allclose(st[k], x, rtol=1e-12, atol=1e-12)


def test_box_signed_distance_brute_force(setup):
    ora, _, _ = setup
    rng = np.random.default_rng(1)
    box = np.array([0.2, 0.3, 0.4, 0.5, 0.45, 0.9], np.float32)
    lo, hi = box[:3].astype(np.float64), box[3:].astype(np.float64)
    for _ in range(200):
        p = rng.uniform(0.0, 1.0, 3)
        inside = np.all(p >= lo) and np.all(p <= hi)
        if inside:
            want = -min(np.min(p - lo), np.min(hi - p))
        else:
            want = np.linalg.norm(p - np.clip(p, lo, hi))
        assert abs(ora.box_sd(box, p) - want) < 1e-12


def test_loss_recomposed_from_states(setup):
    ora, b, D = setup
    boxes = b.problem.boxes.reshape(-1, 6)
    goal = np.asarray(b.problem.goal_center[:3], np.float64)
    for e in range(6):
        n = int(b.n[e])
        L, st = ora.diff_loss(D, b.x0[e], b.u[e], n, states=True)
        sd = np.array([min(ora.box_sd(bx, st[k, :3]) for bx in boxes) for k in range(1, n + 1)])
        z = float(np.float32(50.0)) * (float(np.float32(0.02)) - sd)
        want = (n * float(np.float32(b.dt)) + float(np.float32(0.1)) * np.sum(b.u[e].astype(np.float64) ** 2)
                + np.sum(np.logaddexp(0.0, z)) + np.sum((st[n, :3] - goal) ** 2))
        assert abs(L - want) <= 1e-11 * max(1.0, abs(want))


def test_complex_step_gradient_against_central_differences(setup):
    ora, b, D = setup
    for e in range(4):
        n = int(b.n[e])
        u = b.u[e].astype(np.float64)
        g = ora.diff_grad(D, b.x0[e], u, n)
        fd = np.zeros(16)
        for j in range(16):
            h = 1e-6 * max(1.0, abs(u[j]))
            up, um = u.copy(), u.copy()
            up[j] += h
            um[j] -= h
            fd[j] = (ora.diff_loss(D, b.x0[e], up, n) - ora.diff_loss(D, b.x0[e], um, n)) / (2 * h)
        assert np.linalg.norm(g - fd) <= 1e-6 * np.linalg.norm(g), (g, fd)


def test_gradient_closed_form_without_scene_terms(ora):
    b = W.diff_workload(2, n_edges=4)
    D = ora.DiffProblem(b.problem, b.dt, w_obst=0.0, w_goal=0.0)
    for e in range(4):
        g = ora.diff_grad(D, b.x0[e], b.u[e], int(b.n[e]))
        np.testing.assert_allclose(g, 2 * float(np.float32(0.1)) * b.u[e].astype(np.float64),
                                   rtol=1e-14, atol=1e-14)
