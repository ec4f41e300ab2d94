"""Oracle Quadtree with eps-weighted edges (the tree of the proof of the
uniform-distribution Flowtree upper bound: the edge above a cell of side
2^l weighs 2^(l (1 - eps))) against what the mathematics fixes.

Pins:
* eps = 0 is the plain Quadtree (the exact integer closed form) / 2^Q;
* it is tree W1 under the eps-weighted tree metric: equal to the LP optimum
  with costs t_eps(x, y) summed edge by edge along the path between the two
  leaves (leaf depths and the LCA depth from the exported tree);
* single points: the path weight itself;
* non-increasing in eps (every edge weight 2^(l (1 - eps)) with l >= 0 is).
"""
import numpy as np
import pytest

import gen
import oracle


def world(seed, V=40, d=3, B=30):
    rng = np.random.default_rng(seed)
    X = gen.gaussian_mixture(rng, V, d, 4, 0.3, False)
    return rng, X, oracle.Tree(X, gen.random_shift(rng, d, B), B)


def random_pair(rng, V, s_mu, s_nu, Q):
    mu = rng.choice(V, size=s_mu, replace=False).astype(np.uint32)
    nu = rng.choice(V, size=s_nu, replace=False).astype(np.uint32)

    def masses(n):
        cuts = np.sort(rng.choice(np.arange(1, 1 << Q), size=n - 1, replace=False))
        return np.diff(np.concatenate([[0], cuts, [1 << Q]])).astype(np.uint32)
    return mu, masses(s_mu), nu, masses(s_nu)


def path_weight(T, leaf_depth, x, y, eps):
    if x == y:
        return 0.0
    c = T.lca_depth(int(x), int(y))
    w = lambda k: 2.0 ** ((T.B - k) * (1.0 - eps))
    return sum(w(k) for k in range(c + 1, leaf_depth[x] + 1)) + sum(w(k) for k in range(c + 1, leaf_depth[y] + 1))


@pytest.mark.parametrize("seed", range(6))
def test_eps_zero_is_quadtree(seed):
    rng, X, T = world(seed)
    Q = 12
    mu, mm, nu, nm = random_pair(rng, len(X), 5, 7, Q)
    assert T.quadtree_eps(mu, mm, nu, nm, Q, 0.0) == T.quadtree(mu, mm, nu, nm, Q=Q) / 2.0 ** Q


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("eps", [0.1, 0.35, 0.8])
def test_is_tree_w1_of_the_eps_metric(seed, eps):
    rng, X, T = world(seed)
    Q = 12
    leaf = T.export()["leaf_depth"]
    mu, mm, nu, nm = random_pair(rng, len(X), 4, 6, Q)
    C = np.array([[path_weight(T, leaf, x, y, eps) for y in nu] for x in mu])
    lp = oracle.exact_w1_lp(X, mu, mm, nu, nm, Q, cost=C)
    assert T.quadtree_eps(mu, mm, nu, nm, Q, eps) == pytest.approx(lp, rel=1e-9)


@pytest.mark.parametrize("seed", range(4))
def test_single_points_and_monotone(seed):
    rng, X, T = world(seed)
    leaf = T.export()["leaf_depth"]
    one = [1 << 10]
    for x, y in [(0, 1), (3, 17), (5, 5), (2, 33)]:
        for eps in (0.0, 0.25, 0.5):
            want = path_weight(T, leaf, x, y, eps)
            assert T.quadtree_eps([x], one, [y], one, 10, eps) == pytest.approx(want, rel=1e-12, abs=0)
    Q = 12
    mu, mm, nu, nm = random_pair(rng, len(X), 6, 3, Q)
    vals = [T.quadtree_eps(mu, mm, nu, nm, Q, e) for e in (0.0, 0.2, 0.4, 0.6, 0.8, 1.0)]
    assert all(a >= b for a, b in zip(vals, vals[1:]))
