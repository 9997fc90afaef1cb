"""Pin of the oracle's exclusive scan + GraphSearch (App. A, Alg. 5) on the
paper's worked example, plus brute force on random masks."""

import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "graph_search_example.json")


def test_worked_example(ora):
    g = json.load(open(GOLDEN))
    for case in (g, g["tail_set_case"]):
        S = ora.exclusive_scan(case["mask"])
        assert S.tolist() == case["S"]
        I, count = ora.graph_search(case["mask"], S)
        assert count == case["count"]
        assert I[:count].tolist() == case["I"]


def test_random_masks_against_brute_force(ora):
    rng = np.random.default_rng(0)
    for n in (1, 2, 7, 64, 1000):
        for p in (0.0, 0.1, 0.5, 1.0):
            mask = (rng.random(n) < p).astype(np.uint8)
            S = ora.exclusive_scan(mask)
            I, count = ora.graph_search(mask, S)
            assert count == int(mask.sum())
            assert I[:count].tolist() == list(np.flatnonzero(mask))
            assert S.tolist() == [int(mask[:i].sum()) for i in range(n)]
