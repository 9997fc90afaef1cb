"""Host logic of bench.py (no GPU): the algorithmic byte model, solution-key
costs, time budgets, the gating of committed profile figures on the kernel
sources and the bench arguments, and the one-GPU guard."""

import importlib.util
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


class _Obj:
    def __init__(self, **kw):
        self.__dict__.update(kw)


def test_kernel_bytes_model(bench):
    prob = _Obj(dynamics="QUAD12")
    prm = _Obj(n_cells=1000)
    st = np.zeros(2, dtype=[("n_select", np.int32), ("samples_per_node", np.int32),
                            ("n_survivors", np.int32), ("n_live", np.int64)])
    st["n_select"] = [10, 20]
    st["samples_per_node"] = [32, 32]          # 320 and 640 slots: 2 and 3 tiles of 256
    st["n_survivors"] = [5, 1]
    st["n_live"] = [100, 200]
    kb = bench.kernel_bytes(prob, prm, st)
    d, m = 12, 4
    # prune: regions 9 B, live owners 4 B, survivors 1 B plus 4 B per tile holding one
    np.testing.assert_allclose(kb["prune_flags"], [9000 + 400 + 5 + 2 * 4, 9000 + 800 + 1 + 1 * 4])
    # insert: slots 1 B, tiles 4 B, survivors read 4d + 16 and write 4d + 4m + 28
    per = 4 * d + 16 + 4 * d + 4 * m + 28
    np.testing.assert_allclose(kb["insert"], [320 + 2 * 4 + 5 * per, 640 + 3 * 4 + 1 * per])
    # the close: regions 5 B, the next iteration's selection 4 B each (the last repeats)
    np.testing.assert_allclose(kb["finalize_select"], [5000 + 20 * 4, 5000 + 20 * 4])


def test_key_cost_and_budgets(bench):
    key = (np.uint64(37) << np.uint64(32)) | np.uint64(5)
    assert bench.key_cost(key, "TIME", 0.005) == pytest.approx(37 * 0.005)
    bits = int(np.array([1.25], np.float32).view(np.uint32)[0])
    assert bench.key_cost((bits << 32) | 9, "PATH_LENGTH", 0.005) == 1.25
    assert bench.budgets_for("quad12") == bench.BUDGETS_MS
    assert bench.budgets_for("quad12_paper_small") == bench.BUDGETS_SMALL_DELTA_MS


def test_profile_figures_follow_the_sources_and_the_arguments(bench):
    a = _Obj(workload="quad12", steps=20, warmup=5, iters=200, cost=None, polish=0, polish_goal_only=False,
             cost_first=False, refine_at=0, timing_every=16)
    # the committed summary of `bench.py --gpus 1 --steps 20 --warmup 5` covers the current kernels
    trace, traffic = bench.measured_trace(a), bench.measured_traffic(a)
    assert trace is not None and traffic is not None, "profiles/quad12_* were taken on other kernel sources"
    assert set(trace) == set(bench.KERNELS) and all(v > 0 for v in trace.values())
    assert all(traffic[k] > 0 for k in bench.KERNELS)
    # another window of queries, or another form of the kernels, reads nothing
    assert bench.measured_traffic(_Obj(**dict(vars(a), steps=100))) is None
    assert bench.measured_trace(_Obj(**dict(vars(a), cost_first=True))) is None
    assert bench.measured_trace(_Obj(**dict(vars(a), timing_every=8))) is None  # other bracketed launches


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
