"""Oracle against hand-worked examples (tests/golden/*.json).

Each fixture was derived on paper from Section 2 (tree, weights, closed
form), Appendix A.1 (greedy) and Section 3 (price); see its "derivation".
"""
import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
FIXTURES = ["hand_1d.json", "hand_2d_order.json"]


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


@pytest.mark.parametrize("name", FIXTURES)
def test_tree_matches_hand_derivation(name):
    g = load(name)
    X = np.array(g["X"], np.float32)
    t = oracle.Tree(X, np.array(g["shift"]), g["B"])
    ex = t.export()
    assert ex["code"].tolist() == g["codes"]
    assert ex["rank_of"].tolist() == g["rank_of"]
    assert ex["leaf_depth"].tolist() == g["leaf_depth"]
    for key, val in g["tree_dist"].items():
        a, b = map(int, key.split(","))
        assert t.tree_dist(a, b) == val
        assert t.tree_dist(b, a) == val


@pytest.mark.parametrize("name", FIXTURES)
def test_estimators_match_hand_derivation(name):
    g = load(name)
    X = np.array(g["X"], np.float32)
    t = oracle.Tree(X, np.array(g["shift"]), g["B"])
    Q = g["Q"]
    for c in g["cases"]:
        args = (c["mu_id"], c["mu_m"], c["nu_id"], c["nu_m"])
        assert t.quadtree(*args, Q=Q) == c["quadtree_units"]
        assert t.quadtree_value(*args, Q=Q) == pytest.approx(c["quadtree_value"], rel=1e-12)
        cost, fl = t.flowtree(*args, Q=Q)
        got = [[c["mu_id"][a], c["nu_id"][b], int(e)]
               for a, b, e in zip(fl["mu"], fl["nu"], fl["eta"])]
        assert sorted(got) == sorted(c["flows"])
        assert cost == pytest.approx(c["flowtree"], rel=1e-12)
        w1 = oracle.exact_w1_lp(X, *args, Q=Q)
        assert w1 == pytest.approx(c["w1"], abs=1e-9)
