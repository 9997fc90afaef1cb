"""Adaptive decomposition (kpx_refine) through the C ABI against the float64
oracle: the refined regions, region table, cursor and capacity flag right
after a refinement, and lockstep iterations before and after it."""

import dataclasses

import numpy as np
import pytest

import workloads as W

from oracle import parity

pytestmark = pytest.mark.gpu

CASES = {
    "di6": (dict(n_select=300, samples=9, tree_cap=1 << 16, grid=(8, 8, 8)), 12, 15),
    "quad12": (dict(n_select=260, samples=9, tree_cap=1 << 16, grid=(4, 4, 4)), 12, 15),
}


@pytest.fixture(scope="module")
def kpx():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_02846_amd as K

    K.lib()
    return K


@pytest.mark.parametrize("case", sorted(CASES))
def test_lockstep_across_refinement(kpx, ora, case):
    kw, before, after = CASES[case]
    w = W.make_workload(case, 8, **kw)
    w.params.refine_max = 2
    P = ora.Problem(w.problem, w.params)
    P2 = ora.Problem(w.problem, dataclasses.replace(w.params, grid=tuple(2 * g for g in w.params.grid)))
    pl = kpx.Planner(w.problem, w.params)
    rep = parity.lockstep(ora, P, pl, before)
    assert rep["iterations"] == before
    pre = pl.snapshot()
    pl.refine(2)
    post = pl.snapshot()
    assert pl.n_cells == P2.n_cells and len(post["cell_table"]) == P2.n_cells
    tr = parity.oracle_tree_from_snapshot(ora, P, pre, cells_cap=P2.n_cells)
    assert tr.refine(P2, 2, hint_cell=post["cell"]) == ora.OK
    n = int(post["counters"]["n_tree"])
    np.testing.assert_array_equal(post["cell"], tr.cell[:n])
    np.testing.assert_array_equal(post["status"], tr.status[:n])
    tbl = post["cell_table"]
    reached = tbl != parity.EMPTY
    np.testing.assert_array_equal(reached, tr.tbl_id[: P2.n_cells] >= 0)
    np.testing.assert_array_equal((tbl[reached] & np.uint64(0xFFFFFFFF)).astype(np.int64),
                                  tr.tbl_id[: P2.n_cells][reached])
    assert int(post["counters"]["cursor"]) == int(tr.c.cursor)
    assert int(post["counters"]["full"]) == int(tr.c.full)
    rep2 = parity.lockstep(ora, P2, pl, after)
    print(case, rep, rep2)
    assert rep2["iterations"] == after
    pl.close()


def test_refine_arguments(kpx):
    w = W.make_workload("di6", 0, n_select=64, samples=4, tree_cap=1 << 14, grid=(8, 8, 8))
    pl = kpx.Planner(w.problem, w.params)  # refine_max 0: no refinement
    with pytest.raises(kpx.KPXError):
        pl.refine(2)
    pl.close()
    w.params.refine_max = 4
    pl = kpx.Planner(w.problem, w.params)
    with pytest.raises(kpx.KPXError):
        pl.refine(1)
    with pytest.raises(kpx.KPXError):
        pl.refine(8)  # beyond refine_max
    b = kpx.Batch([pl])
    pl.refine(2)
    with pytest.raises(kpx.KPXError):
        b.iterate(1)  # the batch was made before the refinement
    b.close()
    pl.refine(2)
    with pytest.raises(kpx.KPXError):
        pl.refine(2)  # total factor 8 > 4
    pl.iterate(3)
    assert pl.n_cells == 32 ** 3
    pl.close()
