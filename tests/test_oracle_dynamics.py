"""Pins of the oracle's dynamics and RK4 against closed forms, conservation
laws, rotation-matrix identities and fourth-order convergence."""

import math

import numpy as np
import pytest

import workloads as W


def _P(ora, name, **params):
    w = W.make_workload(name, 0)
    for k, v in params.items():
        setattr(w.problem if hasattr(w.problem, k) else w.params, k, v)
    return ora.Problem(w.problem, w.params), w


# ---------------------------------------------------------------- DI6 ----

def test_di6_rk4_equals_closed_form(ora):
    P, _ = _P(ora, "di6")
    rng = np.random.default_rng(1)
    for _ in range(200):
        x0 = rng.uniform(-1, 1, 6)
        u = rng.uniform(-1, 1, 3)
        n = int(rng.integers(1, 40))
        h = float(np.float32(0.01))
        z = ora.integrate(P, x0, u, n, h)
        T = n * h
        p = x0[:3] + x0[3:] * T + 0.5 * u * T * T
        v = x0[3:] + u * T
        np.testing.assert_allclose(z[:3], p, rtol=0, atol=1e-13)
        np.testing.assert_allclose(z[3:6], v, rtol=0, atol=1e-13)


def test_di6_path_length_closed_form(ora):
    # speed grows linearly along a fixed direction from rest: length = |a| T^2 / 2
    P, _ = _P(ora, "di6")
    u = np.array([0.3, -0.4, 0.0])
    z = ora.integrate(P, np.zeros(6), u, 25, 0.01)
    assert abs(z[6] - 0.5 * 0.5 * 0.25 ** 2) < 1e-14


# ------------------------------------------------------------- QUAD12 ----

def _quad(ora, inertia=(0.01, 0.01, 0.01), mass=1.0, g=9.81):
    w = W.make_workload("quad12", 0)
    w.problem.dyn_params[:5] = np.array([mass, *inertia, g], dtype=np.float32)
    return ora.Problem(w.problem, w.params), w


def _consts(w):
    m, jx, jy, jz, g = (float(v) for v in w.problem.dyn_params[:5])
    return m, np.array([jx, jy, jz]), g


def test_quad_hover_is_a_fixed_point(ora):
    P, w = _quad(ora)
    m, _, g = _consts(w)
    for yaw in (0.0, 0.7, -2.5):
        x0 = np.zeros(12)
        x0[:3] = (0.3, 0.4, 0.5)
        x0[5] = yaw
        z = ora.integrate(P, x0, [m * g, 0, 0, 0], 60, 0.005)
        np.testing.assert_allclose(z[:12], x0, atol=1e-14)


def test_quad_free_fall(ora):
    P, w = _quad(ora)
    _, _, g = _consts(w)
    x0 = np.zeros(12)
    x0[:3] = (0.2, 0.3, 0.9)
    x0[6:9] = (0.1, -0.2, 0.3)
    n, h = 40, 0.005
    z = ora.integrate(P, x0, [0, 0, 0, 0], n, h)
    T = n * h
    np.testing.assert_allclose(z[:3], x0[:3] + x0[6:9] * T - 0.5 * g * T * T * np.array([0, 0, 1]),
                               atol=1e-14)
    np.testing.assert_allclose(z[6:9], x0[6:9] - g * T * np.array([0, 0, 1]), atol=1e-14)


def test_quad_pure_roll(ora):
    P, w = _quad(ora)
    _, J, _ = _consts(w)
    x0 = np.zeros(12)
    x0[3] = 0.1
    x0[9] = 0.5
    tau = 0.3
    n, h = 50, 0.005
    z = ora.integrate(P, x0, [0, tau, 0, 0], n, h)
    T = n * h
    assert abs(z[3] - (0.1 + 0.5 * T + 0.5 * tau / J[0] * T * T)) < 1e-13
    assert abs(z[4]) < 1e-15 and abs(z[5]) < 1e-15
    assert abs(z[9] - (0.5 + tau / J[0] * T)) < 1e-13


def test_quad_isotropic_rates_are_linear_in_time(ora):
    P, w = _quad(ora)
    _, J, _ = _consts(w)
    rng = np.random.default_rng(2)
    x0 = np.zeros(12)
    x0[3:6] = rng.uniform(-0.5, 0.5, 3)
    x0[9:12] = rng.uniform(-2, 2, 3)
    tau = rng.uniform(-0.5, 0.5, 3)
    z = ora.integrate(P, x0, [5.0, *tau], 30, 0.005)
    np.testing.assert_allclose(z[9:12], x0[9:12] + 30 * 0.005 * tau / J, atol=1e-12)


# The path length of the quadrotor, the speed |v| integrated as a 13th RK4
# component (Assumption 1's additive cost; the model is cited in Sec. V).
# Each pin below makes a wrong velocity index, a dropped or doubled component
# or a rate read from another block of the state fail.

def test_quad_path_length_free_fall_from_rest(ora):
    # speed g t grows linearly from rest, which RK4 integrates exactly:
    # length = g T^2 / 2, whatever the (constant) attitude
    P, w = _quad(ora)
    _, _, g = _consts(w)
    x0 = np.zeros(12)
    x0[:3] = (0.5, 0.5, 0.9)
    x0[3:6] = (0.3, -0.2, 1.1)
    n, h = 40, 0.005
    z = ora.integrate(P, x0, [0, 0, 0, 0], n, h)
    T = n * h
    assert abs(z[12] - 0.5 * g * T * T) < 1e-14


def test_quad_path_length_hover_at_constant_velocity(ora):
    # level attitude and thrust m g: the velocity stays put, length = |v| T
    P, w = _quad(ora)
    m, _, g = _consts(w)
    x0 = np.zeros(12)
    x0[:3] = (0.2, 0.6, 0.4)
    x0[5] = 0.7
    x0[6:9] = (0.3, -0.4, 0.5)
    n, h = 50, 0.005
    z = ora.integrate(P, x0, [m * g, 0, 0, 0], n, h)
    T = n * h
    assert abs(z[12] - math.sqrt(0.5) * T) < 1e-14
    np.testing.assert_allclose(z[6:9], x0[6:9], atol=1e-15)


def test_quad_path_length_ballistic_closed_form(ora):
    # thrust off, initial velocity (vx, vy, vz): the horizontal speed c stays
    # constant and the vertical one is vz - g t, so with F(s) =
    # (s sqrt(c^2 + s^2) + c^2 asinh(s / c)) / 2 the length is
    # (F(vz) - F(vz - g T)) / g.  RK4 converges to it at fourth order.
    P, w = _quad(ora)
    _, _, g = _consts(w)
    x0 = np.zeros(12)
    x0[:3] = (0.3, 0.3, 0.5)
    x0[3:6] = (0.1, 0.2, -0.4)
    x0[6:9] = (0.4, -0.3, 0.9)
    c = 0.5

    def F(s):
        return 0.5 * (s * math.sqrt(c * c + s * s) + c * c * math.asinh(s / c))

    T = 0.2
    exact = (F(0.9) - F(0.9 - g * T)) / g
    errs = []
    for n in (10, 20, 40):
        errs.append(abs(ora.integrate(P, x0, [0, 0, 0, 0], n, T / n)[12] - exact))
    assert errs[-1] < 1e-8, errs
    assert 12.0 < errs[0] / errs[1] < 20.0 and 12.0 < errs[1] / errs[2] < 20.0, errs


def _rot(phi, theta, psi):
    cx, sx = math.cos(phi), math.sin(phi)
    cy, sy = math.cos(theta), math.sin(theta)
    cz, sz = math.cos(psi), math.sin(psi)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx  # ZYX (yaw-pitch-roll), body to world


def test_quad_thrust_points_along_body_z(ora):
    P, w = _quad(ora)
    m, _, g = _consts(w)
    rng = np.random.default_rng(3)
    for _ in range(50):
        eta = rng.uniform(-1, 1, 3) * np.array([1, 1, 3])
        x = np.zeros(13)
        x[3:6] = eta
        T = rng.uniform(0, 2 * m * g)
        zdot = ora.deriv(P, x, [T, 0, 0, 0])
        expect = _rot(*eta) @ np.array([0, 0, T / m]) - np.array([0, 0, g])
        np.testing.assert_allclose(zdot[6:9], expect, atol=1e-12)


def test_quad_euler_rates_reproduce_body_rates(ora):
    # with eta' from the model, dR/dt must equal R [w]x (body rates)
    P, _ = _quad(ora)
    rng = np.random.default_rng(4)
    for _ in range(50):
        eta = rng.uniform(-1, 1, 3) * np.array([1, 1, 3])
        w = rng.uniform(-3, 3, 3)
        x = np.zeros(13)
        x[3:6] = eta
        x[9:12] = w
        etadot = ora.deriv(P, x, [0, 0, 0, 0])[3:6]
        eps = 1e-6
        dR = (_rot(*(eta + eps * etadot)) - _rot(*(eta - eps * etadot))) / (2 * eps)
        wx = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
        np.testing.assert_allclose(dR, _rot(*eta) @ wx, atol=1e-7)


def test_quad_torque_free_rigid_body_conserves_momentum_and_energy(ora):
    # anisotropic inertia exercises the gyroscopic terms
    P, w = _quad(ora, inertia=(0.01, 0.02, 0.035))
    _, J, _ = _consts(w)
    x0 = np.zeros(12)
    x0[9:12] = (3.0, -1.5, 2.0)
    z = ora.integrate(P, x0, [0, 0, 0, 0], 2000, 1e-4)
    w0, w1 = x0[9:12], z[9:12]
    assert abs(np.linalg.norm(J * w1) - np.linalg.norm(J * w0)) < 1e-10
    assert abs(0.5 * np.dot(J * w1, w1) - 0.5 * np.dot(J * w0, w0)) < 1e-10
    assert np.linalg.norm(w1 - w0) > 0.1  # the motion is not trivial


# ------------------------------------------------------------ DUBINS6 ----

def test_dubins_straight_line(ora):
    P, _ = _P(ora, "dubins6")
    x0 = np.array([0.1, 0.2, 0.5, 0.4, 0.2, 0.6])
    z = ora.integrate(P, x0, [0, 0, 0], 30, 0.01)
    T = 0.3
    v = 0.6
    np.testing.assert_allclose(z[:3], x0[:3] + v * T * np.array(
        [math.cos(0.4) * math.cos(0.2), math.sin(0.4) * math.cos(0.2), math.sin(0.2)]), atol=1e-14)
    assert abs(z[6] - v * T) < 1e-14


def test_dubins_path_length_with_acceleration(ora):
    P, _ = _P(ora, "dubins6")
    x0 = np.array([0.1, 0.2, 0.5, 0.4, 0.2, 0.6])
    z = ora.integrate(P, x0, [0.5, -0.2, 0.3], 25, 0.01)
    T = 0.25
    assert abs(z[6] - (0.6 * T + 0.5 * 0.3 * T * T)) < 1e-14
    assert abs(z[5] - (0.6 + 0.3 * T)) < 1e-14
    assert abs(z[3] - (0.4 + 0.5 * T)) < 1e-14


def _turn(x0, om, T):
    psi0, gam, v = x0[3], x0[4], x0[5]
    r = v * math.cos(gam) / om
    return np.array([x0[0] + r * (math.sin(psi0 + om * T) - math.sin(psi0)),
                     x0[1] - r * (math.cos(psi0 + om * T) - math.cos(psi0)),
                     x0[2] + v * math.sin(gam) * T])


def test_dubins_coordinated_turn_converges_at_fourth_order(ora):
    P, _ = _P(ora, "dubins6")
    x0 = np.array([0.3, 0.3, 0.4, 0.2, 0.3, 0.8])
    om, T = 0.9, 1.0
    exact = _turn(x0, om, T)
    errs = []
    for n in (10, 20, 40, 80):
        z = ora.integrate(P, x0, [om, 0, 0], n, T / n)
        errs.append(np.abs(z[:3] - exact).max())
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    for r in ratios:
        assert 14.0 < r < 18.0, ratios
    assert errs[-1] < 1e-9


# edge lengths inside RK4's asymptotic range (h * fastest rate well below 1)
# and above the float64 round-off floor
@pytest.mark.parametrize("name,T", [("quad12", 0.1), ("dubins6", 0.4)])
def test_rk4_fourth_order_on_random_edges(ora, name, T):
    P, w = _P(ora, name)
    rng = np.random.default_rng(11)
    lo = w.problem.u_lo[: P.m].astype(float)
    hi = w.problem.u_hi[: P.m].astype(float)
    ratios = []
    for _ in range(100):
        x0 = w.problem.x_init[: P.d].astype(float).copy()
        if name == "quad12":
            x0[3:6] += rng.uniform(-0.5, 0.5, 3)
            x0[6:9] = rng.uniform(-0.5, 0.5, 3)
            x0[9:12] = rng.uniform(-3, 3, 3)
        else:
            x0[3] = rng.uniform(-3, 3)
            x0[4] = rng.uniform(-0.5, 0.5)
            x0[5] = rng.uniform(0.3, 0.9)
        u = rng.uniform(lo, hi)
        ref = ora.integrate(P, x0, u, 64 * 8, T / (64 * 8))[: P.d]
        e1 = np.abs(ora.integrate(P, x0, u, 8, T / 8)[: P.d] - ref).max()
        e2 = np.abs(ora.integrate(P, x0, u, 16, T / 16)[: P.d] - ref).max()
        if e2 > 1e-13:
            ratios.append(e1 / e2)
    ratios = np.array(ratios)
    assert len(ratios) > 80
    assert 14.0 < np.median(ratios) < 18.0, np.median(ratios)
    assert np.mean((ratios > 12) & (ratios < 20)) > 0.9
