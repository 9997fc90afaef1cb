"""Properties of the seeded scene generators (inputs shared by both sides)."""

import numpy as np

import workloads as W


def test_sizes_match_the_benchmark_workloads():
    di, qu, du = (W.make_workload(n, 0) for n in ("di6", "quad12", "dubins6"))
    assert di.problem.n_boxes == 8 and di.params.n_slots == 256 * 8
    assert qu.problem.n_boxes == 64 and qu.params.n_slots == 4096 * 32
    assert qu.params.n_cells == 16 ** 3 * 8 and qu.params.tree_cap == 1 << 21
    assert du.problem.n_boxes == 200 and du.params.n_slots == 8192 * 32
    assert du.params.n_cells == 32 * 32 * 16 and du.params.tree_cap == 1 << 22
    assert di.params.n_cells == 27000


def test_constants_are_float32():
    for n in ("di6", "quad12", "dubins6"):
        w = W.make_workload(n, 1)
        for name in ("dyn_params", "x_init", "x_lo", "x_hi", "u_lo", "u_hi", "ws_lo", "ws_hi",
                     "goal_center", "boxes"):
            assert getattr(w.problem, name).dtype == np.float32
        assert np.float32(w.params.dt) == w.params.dt


def test_boxes_keep_clear_of_start_and_goal():
    for seed in range(10):
        w = W.make_workload("di6", seed)
        b = w.problem.boxes
        s = w.problem.x_init[:3]
        assert not np.any(np.all((b[:, :3] <= s) & (s <= b[:, 3:]), axis=1))
        q = np.clip(w.problem.goal_center, b[:, :3], b[:, 3:])
        assert np.all(np.linalg.norm(q - w.problem.goal_center, axis=1) > w.problem.goal_radius)


def test_wall_has_two_slots():
    for seed in range(5):
        w = W.make_workload("quad12", seed)
        b = w.problem.boxes
        assert np.all(b[:, 0] == np.float32(0.48)) and np.all(b[:, 3] == np.float32(0.52))
        ys = np.linspace(0, 1, 20001)
        covered = np.zeros_like(ys, bool)
        for bb in b[b[:, 2] == 0]:
            covered |= (ys >= bb[1]) & (ys <= bb[4])
        gaps = np.diff(np.concatenate([[0], (~covered).astype(int), [0]]))
        starts, ends = np.flatnonzero(gaps == 1), np.flatnonzero(gaps == -1)
        widths = (ends - starts) * (ys[1] - ys[0])
        assert len(widths) == 2 and np.allclose(widths, 0.08, atol=2e-4)
        # every z layer has the same 8 boxes
        assert b.shape[0] == 64 and len(np.unique(b[:, 2])) == 8


def test_buildings_keep_out_of_start_and_goal():
    w = W.make_workload("dubins6", 0)
    b = w.problem.boxes
    assert np.all(b[:, 2] == 0) and np.all((b[:, 5] >= 0.2) & (b[:, 5] <= 0.9))
    for p in (w.problem.x_init[:2], w.problem.goal_center[:2]):
        q = np.clip(p, b[:, :2], b[:, 3:5])
        assert np.all(np.linalg.norm(q - p, axis=1) >= 0.2 - 1e-6)


def test_seeds_are_reproducible_and_distinct():
    a, b, c = (W.make_workload("dubins6", s).problem.boxes for s in (4, 4, 5))
    assert np.array_equal(a, b) and not np.array_equal(a, c)
