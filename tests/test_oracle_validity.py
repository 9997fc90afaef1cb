"""Pins of the valid set, region map and goal test: brute force on tiny scenes,
the continuous-time truth for the double integrator, and hand-placed points."""

import math

import numpy as np
import pytest

import workloads as W


def _di(ora, boxes, margin=1e-4, **kw):
    w = W.make_workload("di6", 0, **kw)
    w.problem.boxes = np.asarray(boxes, dtype=np.float32).reshape(-1, 6)
    w.problem.margin = float(np.float32(margin))
    return ora.Problem(w.problem, w.params), w


def _brute_first_invalid(ora, P, w, x0, u, n):
    """Direct triple loop: substep x box x axis, against the same float64 states."""
    m = float(w.problem.margin)
    bx = w.problem.boxes.astype(np.float64)
    for k in range(1, n + 1):
        x = ora.integrate(P, x0, u, k)[: P.d]
        p = x[:3]
        if np.any(p < w.problem.ws_lo + m) or np.any(p > w.problem.ws_hi - m):
            return k
        lo, hi = w.problem.x_lo[: P.d].astype(float), w.problem.x_hi[: P.d].astype(float)
        if np.any(x < lo + m) or np.any(x > hi - m):
            return k
        for b in bx:
            inside = True
            for a in range(3):
                if not (b[a] - m <= p[a] <= b[3 + a] + m):
                    inside = False
                    break
            if inside:
                return k
    return 0


def test_collision_brute_force_tiny_scenes(ora):
    rng = np.random.default_rng(5)
    checked = 0
    for scene in range(3):
        nb = scene + 1
        c = rng.uniform(0.3, 0.7, (nb, 3))
        s = rng.uniform(0.05, 0.2, (nb, 3))
        boxes = np.concatenate([c - s / 2, c + s / 2], 1)
        P, w = _di(ora, boxes)
        for _ in range(700):
            x0 = np.concatenate([rng.uniform(0.05, 0.95, 3), rng.uniform(-0.9, 0.9, 3)])
            u = rng.uniform(-1, 1, 3).astype(np.float32)
            n = int(rng.integers(5, 31))
            e = ora.propagate_edge(P, x0, u, n)
            if e["flags"]:
                continue
            assert e["first_invalid"] == _brute_first_invalid(ora, P, w, x0, u.astype(float), n)
            checked += 1
    assert checked > 1900


def _entry_interval(p0, v0, a, lo, hi, T):
    """Times in [0, T] where p0 + v0 t + a t^2 / 2 lies in [lo, hi] (union of
    closed intervals), from the roots of the two quadratics."""
    def roots(c):
        # a/2 t^2 + v0 t + (p0 - c) = 0
        A, B, C = 0.5 * a, v0, p0 - c
        if abs(A) < 1e-300:
            return [] if abs(B) < 1e-300 else [-C / B]
        disc = B * B - 4 * A * C
        if disc < 0:
            return []
        r = math.sqrt(disc)
        return sorted([(-B - r) / (2 * A), (-B + r) / (2 * A)])
    cuts = sorted({0.0, T, *[t for t in roots(lo) + roots(hi) if 0 < t < T]})
    ivs = []
    for t0, t1 in zip(cuts[:-1], cuts[1:]):
        tm = 0.5 * (t0 + t1)
        pm = p0 + v0 * tm + 0.5 * a * tm * tm
        if lo <= pm <= hi:
            ivs.append((t0, t1))
    return ivs


def _intersect(a, b):
    out = []
    for x0, x1 in a:
        for y0, y1 in b:
            lo, hi = max(x0, y0), min(x1, y1)
            if lo <= hi:
                out.append((lo, hi))
    return out


def test_double_integrator_continuous_truth(ora):
    """Per axis the box is entered on intervals given by quadratic roots.  The
    discrete check must flag exactly the first substep time inside them (or an
    earlier bound violation), and may only miss intrusions shorter than one
    substep."""
    rng = np.random.default_rng(9)
    box = np.array([0.4, 0.4, 0.4, 0.6, 0.6, 0.6], dtype=np.float32).astype(float)
    P, w = _di(ora, [box], margin=0.0)
    P0, _ = _di(ora, np.zeros((0, 6)), margin=0.0)  # same problem without the box
    h = float(np.float32(0.01))
    misses = checked = 0
    for _ in range(3000):
        x0 = np.concatenate([rng.uniform(0.2, 0.8, 3), rng.uniform(-0.9, 0.9, 3)])
        u = rng.uniform(-1, 1, 3).astype(np.float32)
        n = 30
        T = n * h
        ivs = [(0.0, T)]
        for a in range(3):
            ivs = _intersect(ivs, _entry_interval(x0[a], x0[3 + a], float(u[a]), box[a], box[3 + a], T))
        ks = [k for k in range(1, n + 1) if any(t0 - 1e-12 <= k * h <= t1 + 1e-12 for t0, t1 in ivs)]
        e = ora.propagate_edge(P, x0, u, n)
        e0 = ora.propagate_edge(P0, x0, u, n)
        if e["flags"] or e0["flags"]:
            continue
        candidates = [k for k in (ks[0] if ks else 0, e0["first_invalid"]) if k]
        assert e["first_invalid"] == (min(candidates) if candidates else 0)
        checked += 1
        if ivs and not ks:
            # an intrusion between substeps: necessarily shorter than one substep
            assert all(t1 - t0 < h for t0, t1 in ivs)
            misses += 1
    assert checked > 2800


def test_closed_boxes_and_closed_bounds(ora):
    P, w = _di(ora, [[0.4, 0.4, 0.4, 0.6, 0.6, 0.6]], margin=0.0)
    face = float(np.float32(0.4))  # the box corner as stored (float32, widened)
    on_face = [face, 0.5, 0.5, 0, 0, 0]
    assert ora.point_status(P, on_face, margin=0.0)[0]  # touching a box face collides
    just_out = [np.nextafter(face, 0), 0.5, 0.5, 0, 0, 0]
    assert not ora.point_status(P, just_out, margin=0.0)[0]
    assert not ora.point_status(P, [0.0, 1.0, 0.2, 1.0, -1.0, 0.0], margin=0.0)[0]  # on bounds: ok
    assert ora.point_status(P, [0.1, 0.1, 0.1, np.nextafter(1.0, 2), 0, 0], margin=0.0)[0]
    assert ora.point_status(P, [-1e-12, 0.1, 0.1, 0, 0, 0], margin=0.0)[0]


def test_margin_grows_boxes_and_shrinks_bounds(ora):
    P, w = _di(ora, [[0.4, 0.4, 0.4, 0.6, 0.6, 0.6]], margin=1e-3)
    m = float(np.float32(1e-3))
    assert ora.point_status(P, [0.4 - m / 2, 0.5, 0.5, 0, 0, 0])[0]
    assert not ora.point_status(P, [0.4 - 2 * m, 0.5, 0.5, 0, 0, 0])[0]
    assert ora.point_status(P, [m / 2, 0.5, 0.2, 0, 0, 0])[0]
    assert ora.point_status(P, [0.2, 0.2, 0.2, 1 - m / 2, 0, 0])[0]


def test_band_flags(ora):
    P, w = _di(ora, [[0.4, 0.4, 0.4, 0.6, 0.6, 0.6]], margin=0.0)
    face = float(np.float32(0.4))
    bad, amb, fl = ora.point_status(P, [face - 5e-6, 0.5, 0.5, 0, 0, 0], margin=0.0, band=1e-5)
    assert not bad and amb and fl == ora.FLAG_BOX
    bad, amb, fl = ora.point_status(P, [face + 5e-6, 0.5, 0.5, 0, 0, 0], margin=0.0, band=1e-5)
    assert bad and amb
    bad, amb, fl = ora.point_status(P, [0.45, 0.5, 0.5, 0, 0, 0], margin=0.0, band=1e-5)
    assert bad and not amb  # deep inside: a clear violation
    bad, amb, fl = ora.point_status(P, [0.2, 0.2, 0.2, 1 - 3e-6, 0, 0], margin=0.0, band=1e-5)
    assert not bad and amb and fl == ora.FLAG_BOUND
    # a clear violation elsewhere overrides a near-threshold check
    bad, amb, fl = ora.point_status(P, [0.45, 0.5, 0.5, 1 - 3e-6, 0, 0], margin=0.0, band=1e-5)
    assert bad and not amb


def test_region_map_hand_placed_points(ora):
    w = W.make_workload("quad12", 0, grid=(4, 5, 2))
    P = ora.Problem(w.problem, w.params)
    def x_at(p, v=(0.1, 0.1, 0.1)):
        x = np.zeros(12)
        x[:3] = p
        x[6:9] = v
        return x
    # cell centres
    c, fl = ora.cell_of(P, x_at((0.125, 0.1, 0.25)))
    assert c == ((0 * 5 + 0) * 2 + 0) * 8 + 7 and fl == 0
    c, _ = ora.cell_of(P, x_at((0.875, 0.9, 0.75), (-0.1, 0.2, -0.3)))
    assert c == ((3 * 5 + 4) * 2 + 1) * 8 + 0b010
    # exactly on an interior face: floor puts it in the upper cell; flagged
    c, fl = ora.cell_of(P, x_at((0.25, 0.1, 0.25)))
    assert c // 8 == (1 * 5 + 0) * 2 + 0 and fl & ora.FLAG_CELL
    # the far workspace face is clamped into the last cell (not flagged)
    c, fl = ora.cell_of(P, x_at((1.0, 1.0, 1.0)))
    assert c // 8 == (3 * 5 + 4) * 2 + 1 and fl == 0
    # velocity exactly 0 counts as non-negative; flagged as near the sign boundary
    c, fl = ora.cell_of(P, x_at((0.125, 0.1, 0.25), (0.0, -0.5, 0.5)))
    assert c % 8 == 0b101 and fl & ora.FLAG_VSIGN
    # a hint is adopted only for an adjacent index across the nearby face
    x = x_at((0.25 + 1e-6, 0.1, 0.25))
    own, _ = ora.cell_of(P, x)
    lower = own - 5 * 2 * 8
    assert ora.cell_of(P, x, hint=lower)[0] == lower
    far = own + 5 * 2 * 8
    assert ora.cell_of(P, x, hint=far)[0] == own


def test_goal_ball(ora):
    w = W.make_workload("di6", 0)
    P = ora.Problem(w.problem, w.params)
    r = float(np.float32(0.05))
    c = w.problem.goal_center.astype(float)
    assert ora.goal_test(P, [*c, 0, 0, 0], radius=r)[0]
    assert ora.goal_test(P, [c[0] + r, c[1], c[2], 0, 0, 0], radius=r)[0]  # closed ball
    assert not ora.goal_test(P, [c[0] + r + 1e-4, c[1], c[2], 0, 0, 0], radius=r)[0]
    inside, fl = ora.goal_test(P, [c[0] + r - 1e-6, c[1], c[2], 0, 0, 0], radius=r)
    assert inside and fl == ora.FLAG_GOAL
