"""Oracle quadtree (Section 2) against brute force from the definition.

The brute force works from the grid codes only: cells at depth k are the
distinct (code >> (B-k)) tuples, a point's leaf is its first cell holding no
other point (depth B at most), and the Morton order is the lexicographic order
of the per-level bit tuples (dimension 0 first).  The codes themselves are
pinned geometrically: every point must lie inside its depth-B cell of the
shifted hypercube H = [-Phi, Phi]^d + sigma around the translated points.
"""
import numpy as np
import pytest

import gen
import oracle


def small_sets():
    out = []
    for seed in range(6):
        rng = np.random.default_rng(100 + seed)
        V = int(rng.integers(2, 48))
        d = int(rng.integers(1, 4))
        B = int(rng.choice([4, 6, 10, 30]))
        X = rng.standard_normal((V, d)).astype(np.float32)
        if seed % 3 == 0:  # coincident points force depth-B multi-point leaves
            X[V // 2] = X[0]
        if seed % 3 == 1:  # clustered points force deep trees
            X = (X * 1e-3 + 5).astype(np.float32)
        out.append((X, gen.random_shift(rng, d, B), B))
    rng = np.random.default_rng(7)
    out.append((gen.pixel_grid(6), gen.random_shift(rng, 2, 30), 30))
    out.append((np.zeros((1, 3), np.float32), np.array([1, 1, 1]), 5))
    out.append((np.ones((4, 2), np.float32), np.array([3, 2]), 6))
    return out


CASES = small_sets()


def brute(code, B):
    V, d = code.shape
    cells = [{} for _ in range(B + 1)]
    for k in range(B + 1):
        for p in range(V):
            key = tuple((code[p] >> (B - k)).tolist())
            cells[k].setdefault(key, []).append(p)
    leaf = np.empty(V, np.int64)
    for p in range(V):
        leaf[p] = B
        for k in range(B + 1):
            if len(cells[k][tuple((code[p] >> (B - k)).tolist())]) == 1:
                leaf[p] = k
                break
    mkey = [tuple(tuple(((code[p] >> (B - k)) & 1).tolist()) for k in range(1, B + 1)) + (p,)
            for p in range(V)]
    order = sorted(range(V), key=lambda p: mkey[p])
    rank = np.empty(V, np.int64)
    rank[order] = np.arange(V)
    nodes = {}
    for k in range(B + 1):
        for key, pts in cells[k].items():
            live = [p for p in pts if leaf[p] >= k]
            if live:
                nodes[(k, key)] = live
    return leaf, rank, nodes, cells


@pytest.mark.parametrize("case", range(len(CASES)))
def test_codes_place_points_in_their_cells(case):
    X, shift, B = CASES[case]
    t = oracle.Tree(X, shift, B)
    ex = t.export()
    code = ex["code"].astype(np.int64)
    assert code.min() >= 0 and code.max() < (1 << B)
    X64 = X.astype(np.float64)
    lo = X64.min(0)
    phi = float((X64.max(0) - lo).max())
    assert t.phi == phi
    if phi == 0:
        assert (code == code[0]).all()
        return
    u = 2 * phi / (1 << B)                        # grid unit
    corner = lo - phi + shift * u                # lower corner of H per dimension
    lo_edge = corner + code * u
    tol = 4e-15 * (1 + np.abs(X64).max()) * (1 << B) * u + 1e-12
    assert (X64 >= lo_edge - tol).all()
    assert (X64 <= lo_edge + u + tol).all()


@pytest.mark.parametrize("case", range(len(CASES)))
def test_tree_structure_brute_force(case):
    X, shift, B = CASES[case]
    t = oracle.Tree(X, shift, B)
    ex = t.export()
    leaf, rank, nodes, _ = brute(ex["code"].astype(np.int64), B)
    assert (ex["leaf_depth"] == leaf).all()
    assert (ex["rank_of"] == rank).all()
    assert t.n_nodes == len(nodes)
    # every node is a contiguous Morton range holding exactly its live points
    pts_by_rank = np.argsort(ex["rank_of"])
    got = {}
    for v in range(t.n_nodes):
        k = int(ex["node_depth"][v])
        members = sorted(pts_by_rank[ex["node_first"][v]:ex["node_last"][v] + 1].tolist())
        got[(k, tuple(sorted(members)))] = True
        if v:
            par = ex["node_parent"][v]
            assert ex["node_depth"][par] == k - 1
            assert ex["node_first"][par] <= ex["node_first"][v] <= ex["node_last"][v] <= ex["node_last"][par]
    want = {(k, tuple(sorted(p))) for (k, _), p in nodes.items()}
    assert set(got) == want


@pytest.mark.parametrize("case", range(len(CASES)))
def test_levels_partition_supports(case):
    """Appendix A.1: the nodes of one level partition the points still
    present at that level."""
    X, shift, B = CASES[case]
    t = oracle.Tree(X, shift, B)
    ex = t.export()
    for k in range(B + 1):
        sel = np.flatnonzero(ex["node_depth"] == k)
        covered = []
        for v in sel:
            covered += list(range(ex["node_first"][v], ex["node_last"][v] + 1))
        live = np.sort(ex["rank_of"][ex["leaf_depth"] >= k])
        assert sorted(covered) == live.tolist()


@pytest.mark.parametrize("case", range(len(CASES)))
def test_tree_distance(case):
    """t(x, y) = sum of side lengths on the leaf-to-leaf path (Section 2);
    both points lie in their common cell, so ||x - y||_inf <= t(x, y)."""
    X, shift, B = CASES[case]
    t = oracle.Tree(X, shift, B)
    ex = t.export()
    leaf, _, _, cells = brute(ex["code"].astype(np.int64), B)
    code = ex["code"].astype(np.int64)
    V = len(X)
    u = t.grid_unit()
    for x in range(min(V, 12)):
        for y in range(V):
            L = max(k for k in range(B + 1) if ((code[x] >> (B - k)) == (code[y] >> (B - k))).all())
            L = min(L, leaf[x], leaf[y])
            want = sum(1 << (B - k) for k in range(L + 1, leaf[x] + 1)) + \
                sum(1 << (B - k) for k in range(L + 1, leaf[y] + 1))
            assert t.tree_dist(x, y) == want
            assert t.lca_depth(x, y) == L
            if x != y and t.phi > 0:
                assert np.abs(X[x].astype(float) - X[y]).max() <= (1 << (B - L)) * u * (1 + 1e-12)


def test_workload_tree_sizes():
    ds = gen.make("tiny")
    t = oracle.Tree(ds.X, ds.shift, ds.B)
    ex = t.export()
    assert sorted(ex["rank_of"].tolist()) == list(range(ds.V))
    assert 2 <= ex["leaf_depth"].max() <= ds.B
