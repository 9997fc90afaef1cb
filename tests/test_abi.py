"""The C-ABI library loads, exports every function include/kpx.h declares, and
rejects invalid problems on the host (no GPU call is made on those paths)."""

import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def kpx():
    import paper_2602_02846_amd as K

    K.lib()
    return K


def declared_functions():
    text = open(os.path.join(ROOT, "include", "kpx.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(kpx_\w+)\s*\(", text, re.M)))


def test_every_declared_symbol_is_exported(kpx):
    names = declared_functions()
    assert len(names) >= 18
    lib = ctypes.CDLL(kpx.kpx.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(kpx):
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        assert kpx.status_string(code) not in ("", "unknown status")
    assert kpx.status_string(99) == "unknown status"


def test_workspace_bytes_hold_the_refined_regions(kpx):
    a = W.make_workload("quad12", 0)
    b = W.make_workload("quad12", 0)
    b.params.refine_max = 2
    na = kpx.workspace_bytes(a.problem, a.params)
    nb = kpx.workspace_bytes(b.problem, b.params)
    # the region table (8 B), activity byte and block counts for 8x the regions
    assert nb - na >= 7 * a.params.n_cells * 9


def test_workspace_bytes_scale_with_capacity(kpx):
    a = W.make_workload("quad12", 0)
    b = W.make_workload("quad12", 0, tree_cap=1 << 22)
    na = kpx.workspace_bytes(a.problem, a.params)
    nb = kpx.workspace_bytes(b.problem, b.params)
    assert nb > na > 0
    # per node: 12 + 4 floats, steps, parent, cost, cell and three status bytes
    assert (nb - na) >= (1 << 21) * (16 * 4 + 2 + 4 * 3 + 3)


def _bad(kpx, name="di6", edit=None, **kw):
    w = W.make_workload(name, 0, **kw)
    if edit:
        edit(w)
    return kpx.kpx.create_status(w.problem, w.params)


def test_invalid_arguments_are_rejected(kpx):
    ERR_ARG, ERR_START = -1, -2
    assert _bad(kpx, edit=lambda w: setattr(w.params, "steps_min", 0)) == ERR_ARG
    assert _bad(kpx, edit=lambda w: setattr(w.params, "n_select", 0)) == ERR_ARG
    assert _bad(kpx, edit=lambda w: setattr(w.params, "i_max", 255)) == ERR_ARG
    assert _bad(kpx, edit=lambda w: setattr(w.params, "dt", 0.0)) == ERR_ARG
    assert _bad(kpx, tree_cap=2048) == ERR_ARG  # < 1 + 2048 survivors
    assert _bad(kpx, "dubins6", edit=lambda w: setattr(w.params, "vel_sign_bins", 1)) == ERR_ARG
    assert _bad(kpx, edit=lambda w: setattr(w.problem, "goal_radius", 1e-5)) == ERR_ARG

    def flip_box(w):
        w.problem.boxes[0, 0], w.problem.boxes[0, 3] = w.problem.boxes[0, 3], w.problem.boxes[0, 0]
    assert _bad(kpx, edit=flip_box) == ERR_ARG

    def start_in_box(w):
        w.problem.x_init[:3] = (w.problem.boxes[0, :3] + w.problem.boxes[0, 3:]) / 2
    assert _bad(kpx, edit=start_in_box) == ERR_START

    def start_too_fast(w):
        w.problem.x_init[3] = 1.0  # on the bound, inside the clearance margin
    assert _bad(kpx, edit=start_too_fast) == ERR_START
    assert _bad(kpx, edit=lambda w: setattr(w.params, "refine_max", 9)) == ERR_ARG
    def refine_too_far(w):  # 256^3 regions refined 8x per axis exceed 2^30 regions
        w.params.grid = (256, 256, 256)
        w.params.refine_max = 8
    assert _bad(kpx, edit=refine_too_far) == ERR_ARG


def test_null_arguments(kpx):
    L = kpx.lib()
    assert L.kpx_create(None, None, None, None, 0, None) == -1
    assert L.kpx_iterate(None, 1) == -1
    assert L.kpx_destroy(None) == 0
    out = ctypes.c_size_t(0)
    assert L.kpx_workspace_bytes(None, None, ctypes.byref(out)) == -1
    assert L.kpx_batch_create(None, 0, None) == -1
    assert L.kpx_batch_set_graph(None, 1) == -1
    assert L.kpx_batch_iterate(None, 1) == -1
    assert L.kpx_batch_destroy(None) == 0
    assert L.kpx_refine(None, 2) == -1
    assert L.kpx_set_polish(None, None) == -1
    assert L.kpx_set_timing_every(None, 1) == -1
    assert L.kpx_set_cost_first(None, 1) == -1
    assert L.kpx_batch_set_threads(None, 0, 256) == -1


def test_diff_invalid_arguments_are_rejected(kpx):
    from paper_2602_02846_amd import diff

    w = W.make_workload("quad12", 0)
    dt = w.params.dt

    def status(edit=None, dt=dt):
        ww = W.make_workload("quad12", 0)
        if edit:
            edit(ww.problem)
        return diff.create_status(ww.problem, dt)

    assert status(dt=0.0) == -1
    assert status(lambda p: p.dyn_params.__setitem__(0, 0.0)) == -1  # mass
    assert status(lambda p: p.dyn_params.__setitem__(2, -1.0)) == -1  # inertia

    def flip_u(p):
        p.u_lo[1], p.u_hi[1] = p.u_hi[1], p.u_lo[1]
    assert status(flip_u) == -1

    def flip_box(p):
        p.boxes[3, 1], p.boxes[3, 4] = p.boxes[3, 4], p.boxes[3, 1]
    assert status(flip_box) == -1

    def many_boxes(p):
        p.boxes = np.tile(p.boxes, (1025 // len(p.boxes) + 1, 1))[:1025]
    assert status(many_boxes) == -1


def test_diff_null_arguments(kpx):
    from paper_2602_02846_amd import diff

    L = diff._lib()
    assert L.kpx_diff_create(None, None, None) == -1
    assert L.kpx_diff_loss_grad(None, None, None, None, 1, None, None) == -1
    assert L.kpx_diff_polish(None, None, None, None, 1, 1, 0.1, None, None) == -1
    assert L.kpx_diff_destroy(None) == 0
    assert L.kpx_diff_last_error(None) == b""
