"""Pins of the oracle's Philox4x32-10 and of the control/duration sample map.

The oracle's block function is checked against rocRAND's host-callable
Philox4x32-10 engine (an independent implementation shipped with ROCm).
"""

import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc")
    if hipcc is None or not os.path.isdir("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available")
    out = tmp_path_factory.mktemp("philox") / "ref"
    subprocess.check_call([hipcc, "-O1", "-std=c++17", "-o", str(out),
                           os.path.join(HERE, "rocrand_philox_ref.cpp")])
    return str(out)


def test_philox_matches_rocrand(ora, rocrand_ref):
    rng = np.random.default_rng(7)
    cases = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF,) * 6, (1, 2, 3, 4, 5, 6)]
    cases += [tuple(int(v) for v in rng.integers(0, 2**32, size=6, dtype=np.uint64))
              for _ in range(2000)]
    # the sample contract's counters: (iteration, slot, query, block)
    cases += [(it, s, 0, b, 12345, 0) for it in (0, 1, 199) for s in (0, 1, 131071) for b in (0, 1)]
    text = "".join(" ".join(str(v) for v in c) + "\n" for c in cases)
    res = subprocess.run([rocrand_ref], input=text, capture_output=True, text=True, check=True)
    ref = np.array([[int(v) for v in line.split()] for line in res.stdout.strip().splitlines()],
                   dtype=np.uint64)
    assert ref.shape == (len(cases), 4)
    mine = np.array([ora.philox(c[:4], c[4:]) for c in cases], dtype=np.uint64)
    np.testing.assert_array_equal(mine, ref)


def test_philox_is_a_bijection_sample(ora):
    # distinct counters under one key give distinct blocks (a permutation)
    outs = {tuple(ora.philox((i, 0, 0, 0), (99, 1))) for i in range(4096)}
    assert len(outs) == 4096


def _problem(ora, name="quad12", **kw):
    w = W.make_workload(name, 3, **kw)
    return ora.Problem(w.problem, w.params), w


def test_sample_map_uses_the_stated_words(ora):
    P, w = _problem(ora)
    key = (w.params.seed & 0xFFFFFFFF, w.params.seed >> 32)
    for it, slot in [(0, 0), (5, 77), (199, 131071)]:
        u, n = ora.sample(P, it, slot)
        words = np.concatenate([ora.philox((it, slot, 0, 0), key), ora.philox((it, slot, 0, 1), key)])
        lo = w.problem.u_lo.astype(np.float32)
        hi = w.problem.u_hi.astype(np.float32)
        m = P.m
        for i in range(m):
            unit = np.float32(int(words[i]) >> 8) * np.float32(2.0 ** -24)
            # fma with a single rounding: exact product+sum in float64, then round once
            expect = np.float32(float(unit) * float(np.float32(hi[i] - lo[i])) + float(lo[i]))
            assert u[i] == expect
        span = w.params.steps_max - w.params.steps_min + 1
        assert n == w.params.steps_min + ((int(words[m]) * span) >> 32)


def test_samples_lie_in_the_control_box_and_step_range(ora):
    for name in ("di6", "quad12", "dubins6"):
        P, w = _problem(ora, name)
        us, ns = [], []
        for s in range(3000):
            u, n = ora.sample(P, 1, s)
            us.append(u[: P.m])
            ns.append(n)
        us, ns = np.array(us), np.array(ns)
        assert np.all(us >= w.problem.u_lo[: P.m]) and np.all(us <= w.problem.u_hi[: P.m])
        assert ns.min() >= w.params.steps_min and ns.max() <= w.params.steps_max
        # every step count is reachable and roughly uniform (chi-square, loose)
        span = w.params.steps_max - w.params.steps_min + 1
        counts = np.bincount(ns - w.params.steps_min, minlength=span)
        expect = len(ns) / span
        chi2 = ((counts - expect) ** 2 / expect).sum()
        assert chi2 < span + 6 * np.sqrt(2 * span)
        # controls are uniform over the box: mean near the centre
        centre = (w.problem.u_lo[: P.m] + w.problem.u_hi[: P.m]) / 2
        width = w.problem.u_hi[: P.m] - w.problem.u_lo[: P.m]
        assert np.all(np.abs(us.mean(0) - centre) < 0.05 * width)


def test_samples_depend_on_every_counter_field(ora):
    P, w = _problem(ora, "di6")
    base = ora.sample(P, 3, 10)
    assert not np.array_equal(ora.sample(P, 4, 10)[0], base[0])
    assert not np.array_equal(ora.sample(P, 3, 11)[0], base[0])
    w2 = W.make_workload("di6", 3)
    w2.params.query_id = 1
    P2 = ora.Problem(w2.problem, w2.params)
    assert not np.array_equal(ora.sample(P2, 3, 10)[0], base[0])
