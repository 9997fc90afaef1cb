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


def _edge(b, v0, thrust):
    """An edge from a level hover state at (0.5, 0.5, 0.5) with velocity v0 and
    a constant control (thrust, zero torques) in all four segments."""
    x0 = np.zeros(12)
    x0[:3] = 0.5
    x0[6:9] = v0
    u = np.tile(np.array([thrust, 0.0, 0.0, 0.0]), 4)
    return x0, u


def test_path_length_at_constant_velocity(ora):
    """Level hover thrust (T = m g) and zero torques keep a horizontal
    velocity constant: the path length is |v| n dt."""
    b = W.diff_workload(0, n_edges=1)
    D = ora.DiffProblem(b.problem, b.dt, w_ctrl=0.0, w_obst=0.0, w_goal=0.0, w_len=1.0)
    m, g = float(np.float32(b.problem.dyn_params[0])), float(np.float32(b.problem.dyn_params[4]))
    dt = float(np.float32(b.dt))
    for v0, n in (((0.3, -0.4, 0.0), 20), ((0.0, 0.7, 0.0), 33)):
        x0, u = _edge(b, v0, m * g)
        L = ora.diff_loss(D, x0, u, n)
        assert abs((L - n * dt) - np.linalg.norm(v0) * n * dt) <= 1e-13


def test_path_length_in_free_fall(ora):
    """Zero thrust from rest: |v| = g t, so the length is g T^2 / 2, which
    the RK4 steps integrate exactly."""
    b = W.diff_workload(0, n_edges=1)
    D = ora.DiffProblem(b.problem, b.dt, w_ctrl=0.0, w_obst=0.0, w_goal=0.0, w_len=2.5)
    g = float(np.float32(b.problem.dyn_params[4]))
    dt = float(np.float32(b.dt))
    for n in (7, 30):
        x0, u = _edge(b, (0.0, 0.0, 0.0), 0.0)
        L = ora.diff_loss(D, x0, u, n)
        T = n * dt
        assert abs((L - T) / 2.5 - 0.5 * g * T * T) <= 1e-13


def test_path_length_gradient_against_central_differences(ora):
    b = W.diff_workload(3, n_edges=4)
    D = ora.DiffProblem(b.problem, b.dt, w_len=3.0)
    D0 = ora.DiffProblem(b.problem, b.dt, w_len=0.0)
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
        # the length term changes the gradient (it is not silently dropped)
        assert np.linalg.norm(g - ora.diff_grad(D0, b.x0[e], u, n)) > 1e-3 * np.linalg.norm(g)


def test_path_length_matches_the_planner_oracle(ora):
    """The rollout's length term equals the planner oracle's path-length cost
    of the same edge (one control for all segments)."""
    w = W.make_workload("quad12", 0, cost="PATH_LENGTH")
    P = ora.Problem(w.problem, w.params)
    b = W.diff_workload(4, n_edges=6)
    D = ora.DiffProblem(b.problem, b.dt, w_ctrl=0.0, w_obst=0.0, w_goal=0.0, w_len=1.0)
    dt = float(np.float32(b.dt))
    assert dt == float(np.float32(w.params.dt))
    for e in range(6):
        n = int(b.n[e])
        u4 = b.u[e, :4].astype(np.float64)
        L = ora.diff_loss(D, b.x0[e], np.tile(u4, 4), n)
        length = ora.integrate(P, b.x0[e].astype(np.float64), u4, n)[12]  # the path-length component
        assert length > 0.0
        assert abs((L - n * dt) - length) <= 1e-12 * max(1.0, length)
