"""Oracle Quadtree / Flowtree / exact W1 against what the paper and the
mathematics fix, on tiny inputs.

Pins:
* Quadtree closed form == optimum of the transport LP under the tree metric
  (Section 2: the closed form IS tree W1), exactly, as integers.
* Flowtree's flow: marginals exact (Section 3: a coupling of mu and nu); its
  tree cost equals the Quadtree value (the greedy is tree-optimal, Appendix
  A.1); at most |supp mu| + |supp nu| - 1 pairs (every match exhausts one
  side, Appendix A.1).
* Flowtree value: >= exact W1 (its flow is feasible, proof of the Flowtree
  upper bound); inside [min, max] of the Euclidean price over all
  tree-optimal couplings (the LP bracket); 0 on identical inputs; the plain
  distance for single points.
* Random model (Section 3.2, proof of the random-model theorem): when every
  smallest common cell H_k of (x_k, y_k) holds no other planted x, Flowtree
  equals the planted matching cost exactly.
* Exact W1: LP, successive shortest paths and permutations agree.
"""
import numpy as np
import pytest

import gen
import oracle


def random_pair(rng, V, s_mu, s_nu, Q, shared=0):
    mu = rng.choice(V, size=s_mu, replace=False)
    nu = rng.choice(V, size=s_nu, replace=False)
    if shared:
        nu[:shared] = mu[:shared]
        nu = np.unique(nu)
        while len(nu) < s_nu:
            extra = rng.integers(0, V)
            if extra not in nu:
                nu = np.append(nu, extra)
    def masses(n):
        cuts = np.sort(rng.choice(np.arange(1, 1 << Q), size=n - 1, replace=False))
        return np.diff(np.concatenate([[0], cuts, [1 << Q]])).astype(np.uint32)
    return mu.astype(np.uint32), masses(s_mu), nu.astype(np.uint32), masses(s_nu)


def tiny_world(seed, V=40, d=3, B=30):
    rng = np.random.default_rng(seed)
    X = gen.gaussian_mixture(rng, V, d, 4, 0.3, False)
    return rng, X, oracle.Tree(X, gen.random_shift(rng, d, B), B)


CASES = [(seed, s_mu, s_nu, shared) for seed in range(8) for (s_mu, s_nu, shared) in
         [(1, 1, 0), (3, 5, 0), (6, 6, 2), (8, 4, 3)]]


@pytest.mark.parametrize("seed,s_mu,s_nu,shared", CASES)
def test_quadtree_is_tree_w1(seed, s_mu, s_nu, shared):
    rng, X, t = tiny_world(seed)
    Q = 12
    mu_id, mu_m, nu_id, nu_m = random_pair(rng, len(X), s_mu, s_nu, Q, shared)
    U = t.quadtree(mu_id, mu_m, nu_id, nu_m, Q=Q)
    lp = oracle.tree_w1_lp(t, mu_id, mu_m, nu_id, nu_m, Q)
    assert U == round(lp * (1 << Q))
    assert abs(U - lp * (1 << Q)) < 1e-6 * max(1.0, U)


@pytest.mark.parametrize("seed,s_mu,s_nu,shared", CASES)
def test_flow_properties(seed, s_mu, s_nu, shared):
    rng, X, t = tiny_world(seed)
    Q = 12
    mu_id, mu_m, nu_id, nu_m = random_pair(rng, len(X), s_mu, s_nu, Q, shared)
    cost, fl = t.flowtree(mu_id, mu_m, nu_id, nu_m, Q=Q)
    E = len(fl["eta"])
    # a coupling: exact integer marginals
    assert np.bincount(fl["mu"], weights=fl["eta"], minlength=s_mu).astype(np.int64).tolist() == mu_m.astype(np.int64).tolist()
    assert np.bincount(fl["nu"], weights=fl["eta"], minlength=s_nu).astype(np.int64).tolist() == nu_m.astype(np.int64).tolist()
    assert (fl["eta"] > 0).all()
    # each match exhausts a side -> at most s_mu + s_nu - 1 distinct pairs
    assert E <= s_mu + s_nu - 1
    assert len({(a, b) for a, b in zip(fl["mu"], fl["nu"])}) == E
    # tree-optimal: tree cost of the flow equals the closed form
    tc = sum(int(e) * t.tree_dist(mu_id[a], nu_id[b]) for a, b, e in zip(fl["mu"], fl["nu"], fl["eta"]))
    assert tc == t.quadtree(mu_id, mu_m, nu_id, nu_m, Q=Q)
    # the price is the Euclidean cost of that flow, >= W1, inside the bracket
    w1 = oracle.exact_w1_lp(X, mu_id, mu_m, nu_id, nu_m, Q=Q)
    assert cost >= w1 - 1e-9
    lo, hi = oracle.flow_face_bracket(t, mu_id, mu_m, nu_id, nu_m, Q)
    assert lo - 1e-7 <= cost <= hi + 1e-7
    # bind codes say which side the match used up
    rm = mu_m.astype(np.int64).copy()
    rn = nu_m.astype(np.int64).copy()
    for a, b, e, bind in zip(fl["mu"], fl["nu"], fl["eta"], fl["bind"]):
        assert e == min(rm[a], rn[b])
        rm[a] -= e
        rn[b] -= e
        assert bind == (2 if rm[a] == 0 and rn[b] == 0 else (0 if rm[a] == 0 else 1))


@pytest.mark.parametrize("seed", range(6))
def test_identity_symmetry_triangle(seed):
    rng, X, t = tiny_world(seed)
    Q = 10
    a = random_pair(rng, len(X), 5, 4, Q)
    b = random_pair(rng, len(X), 3, 6, Q)
    A, Bd, C = (a[0], a[1]), (a[2], a[3]), (b[0], b[1])
    assert t.quadtree(*A, *A, Q=Q) == 0
    c0, fl = t.flowtree(*A, *A, Q=Q)
    assert c0 == 0.0
    assert t.quadtree(*A, *Bd, Q=Q) == t.quadtree(*Bd, *A, Q=Q)
    assert t.quadtree(*A, *C, Q=Q) <= t.quadtree(*A, *Bd, Q=Q) + t.quadtree(*Bd, *C, Q=Q)
    # swapping the roles of mu and nu transposes the flow (matching is symmetric)
    c1, f1 = t.flowtree(*A, *Bd, Q=Q)
    c2, f2 = t.flowtree(*Bd, *A, Q=Q)
    assert c1 == c2
    assert f1["mu"].tolist() == f2["nu"].tolist() and f1["nu"].tolist() == f2["mu"].tolist()
    assert f1["eta"].tolist() == f2["eta"].tolist()


@pytest.mark.parametrize("seed", range(6))
def test_single_points(seed):
    rng, X, t = tiny_world(seed)
    Q = 20
    for _ in range(10):
        x, y = map(int, rng.choice(len(X), 2, replace=False))
        m = [1 << Q]
        assert t.quadtree([x], m, [y], m, Q=Q) == t.tree_dist(x, y) << Q
        c, fl = t.flowtree([x], m, [y], m, Q=Q)
        assert c == pytest.approx(np.linalg.norm(X[x].astype(float) - X[y]), rel=1e-14)
        assert oracle.exact_w1_ssp(X, [x], m, [y], m, Q) == pytest.approx(c, rel=1e-14)


@pytest.mark.parametrize("seed", range(10))
def test_exact_w1_three_ways(seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((30, 4)).astype(np.float32)
    for s in (2, 4):  # uniform equal sizes with exact masses 2^Q / s
        Q = 8
        mu = rng.choice(30, s, replace=False)
        nu = rng.choice(30, s, replace=False)
        m = np.full(s, (1 << Q) // s, np.uint32)
        lp = oracle.exact_w1_lp(X, mu, m, nu, m, Q=Q)
        ssp = oracle.exact_w1_ssp(X, mu, m, nu, m, Q)
        br = oracle.exact_w1_brute(X, mu, nu)
        assert lp == pytest.approx(br, rel=1e-9, abs=1e-12)
        assert ssp == pytest.approx(br, rel=1e-12, abs=1e-12)
    for s in (3, 5, 7):  # permutations against the LP with exact 1/s weights
        mu = rng.choice(30, s, replace=False)
        nu = rng.choice(30, s, replace=False)
        w = np.full(s, 1.0 / s)
        assert oracle.exact_w1_lp(X, mu, w, nu, w) == pytest.approx(oracle.exact_w1_brute(X, mu, nu), rel=1e-9)
    Q = 10
    a = random_pair(rng, 30, 6, 5, Q)
    assert oracle.exact_w1_ssp(X, *a, Q) == pytest.approx(oracle.exact_w1_lp(X, *a, Q=Q), rel=1e-9)


@pytest.mark.parametrize("seed,eps", [(s, e) for s in range(20) for e in (0.25, 0.05)])
def test_random_model_exactness(seed, eps):
    """Random model with d = 10, s = 8 (the paper's d, with s a power of two
    so uniform masses are exact): under the event of the proof, the tree
    flow is the planted matching and Flowtree is exact."""
    rng = np.random.default_rng(1000 + seed)
    N, d, s, Q = 300, 10, 8, 24
    X, doc, qry = gen.random_model(rng, N, d, s, eps)
    t = oracle.Tree(X, gen.random_shift(rng, d, 30), 30)
    m = np.full(s, (1 << Q) // s, np.uint32)
    Hk = [t.lca_depth(doc[k], qry[k]) for k in range(s)]
    event = all(t.lca_depth(doc[j], doc[k]) < Hk[k] for k in range(s) for j in range(s) if j != k)
    cost, fl = t.flowtree(doc, m, qry, m, Q=Q)
    planted = float(np.mean([np.linalg.norm(X[doc[k]].astype(float) - X[qry[k]]) for k in range(s)]))
    if event:
        assert sorted(zip(fl["mu"].tolist(), fl["nu"].tolist())) == [(k, k) for k in range(s)]
        assert cost == pytest.approx(planted, rel=1e-13)
    assert cost >= planted - 1e-12 or cost >= oracle.exact_w1_lp(X, doc, m, qry, m, Q=Q) - 1e-9


def test_random_model_event_occurs():
    """The exactness test above must see the event often enough to mean
    something (eps = 0.05 makes it frequent)."""
    hits = 0
    for seed in range(20):
        rng = np.random.default_rng(1000 + seed)
        X, doc, qry = gen.random_model(rng, 300, 10, 8, 0.05)
        t = oracle.Tree(X, gen.random_shift(rng, 10, 30), 30)
        Hk = [t.lca_depth(doc[k], qry[k]) for k in range(8)]
        hits += all(t.lca_depth(doc[j], doc[k]) < Hk[k] for k in range(8) for j in range(8) if j != k)
    assert hits >= 5


def test_topk_order():
    rng = np.random.default_rng(0)
    keys = rng.integers(0, 20, 200)
    ids = rng.permutation(200)
    k, i = oracle.topk(keys, ids, 17)
    want = sorted(zip(keys.tolist(), ids.tolist()))[:17]
    assert list(zip(k.tolist(), i.tolist())) == want


def test_invalid_inputs_rejected():
    rng, X, t = tiny_world(0)
    Q = 4
    with pytest.raises(oracle.OracleError):
        t.quadtree([0, 1], [8, 7], [2], [16], Q=Q)      # mass does not sum to 2^Q
    with pytest.raises(oracle.OracleError):
        t.flowtree([0, 0], [8, 8], [2], [16], Q=Q)      # duplicate id
    with pytest.raises(oracle.OracleError):
        t.flowtree([len(X)], [16], [2], [16], Q=Q)      # id out of range
    with pytest.raises(oracle.OracleError):
        t.flowtree([0, 1], [16, 0], [2], [16], Q=Q)     # zero mass
