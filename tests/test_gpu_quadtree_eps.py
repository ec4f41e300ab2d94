"""HIP eps-weighted Quadtree (ft_quadtree_eps_pairs / ft_quadtree_eps_knn)
against the CPU oracle, through the C ABI.

The eps-weighted tree is the one of the proof of the uniform-distribution
Flowtree bound (Appendix A): the edge above a cell of side 2^l weighs
2^(l (1 - eps)).  Bars: float64 pair values within 1e-12 of the oracle,
relative to the largest value a pair can take on this tree (the GPU sums
signed per-cell terms, the oracle sums |mu(v) - nu(v)|, so the two differ by
rounding only); float32 top-k values within 1e-5 relative and the identical
ordered top-k up to near-ties (2e-5 relative); eps = 0 equals the integer
Quadtree key / 2^Q.
"""
import math
import sys

import numpy as np
import pytest

import gen
from gpu_util import build_index, check_topk, oracle_tree, queries, t

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL_SCALE = 1e-12


@pytest.fixture(scope="module")
def ft():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_04126_amd as m
    m.load()
    return m


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def value_scale(B, eps):
    """Largest eps-Quadtree value of two unit-mass distributions: both send
    all their mass through every level, 2 sum_{k=1..B} 2^((B-k)(1-eps))."""
    return 2.0 * sum(2.0 ** ((B - k) * (1.0 - eps)) for k in range(1, B + 1))


def oracle_pairs(T, ds, pq, pd, eps):
    out = np.empty(len(pq))
    for i, (q, d) in enumerate(zip(pq, pd)):
        mu = slice(ds.doc_off[d], ds.doc_off[d + 1])
        nu = slice(ds.q_off[q], ds.q_off[q + 1])
        out[i] = T.quadtree_eps(ds.doc_id[mu], ds.doc_mass[mu], ds.q_id[nu], ds.q_mass[nu], ds.Q, eps)
    return out


def small_world(case):
    """A ground set with coincident points and a tight cluster (deep tree),
    the 28 x 28 pixel grid (many equal values) and a shallow B = 8 grid."""
    rng = np.random.default_rng(5)
    if case == "dup_cluster":
        X = rng.standard_normal((300, 3)).astype(np.float32)
        X[100:110] = X[0]
        X[200:260] = (X[200:260] * 1e-4 + 3).astype(np.float32)
        return X, gen.random_shift(rng, 3, 30), 30
    if case == "grid28":
        return gen.pixel_grid(28), gen.random_shift(rng, 2, 30), 30
    return rng.standard_normal((200, 2)).astype(np.float32), gen.random_shift(rng, 2, 8), 8


def dataset_on(X, shift, B, n_docs, n_q, lo, hi, Q, seed):
    rng = np.random.default_rng(seed)
    V = len(X)

    def dists(n):
        sizes = rng.integers(lo, min(hi, V) + 1, size=n)
        off = np.zeros(n + 1, np.int64)
        off[1:] = np.cumsum(sizes)
        ids = np.concatenate([rng.choice(V, s, replace=False) for s in sizes]).astype(np.uint32)
        return off, ids, gen.uniform_masses(off, ids, Q)

    do, di, dm = dists(n_docs)
    qo, qi, qm = dists(n_q)
    return gen.Dataset("custom", X, np.asarray(shift, np.int64), B, Q, do, di, dm, qo, qi, qm, 5)


def check_pairs(ft, ds, ix, T, pq, pd, eps):
    got = ft.quadtree_eps_pairs(ix, *queries(ds), t(pq), t(pd), eps).cpu().numpy()
    want = oracle_pairs(T, ds, pq, pd, eps)
    tol = REL_SCALE * value_scale(ds.B, eps)
    err = np.abs(got - want)
    assert err.max() <= tol, "eps %.3f: max |gpu - oracle| %.3e > %.3e" % (eps, err.max(), tol)
    return got, want


@pytest.mark.parametrize("eps", [0.0, 0.25, 1.0 / math.log2(30), 0.7, 1.0])
def test_eps_pairs_tiny_all(ft, eps):
    ds = gen.make("tiny")
    say("quadtree eps pairs: tiny, all %d pairs, eps %.3f" % (ds.n_queries * ds.n_docs, eps))
    ix = build_index(ft, ds)
    T = oracle_tree(ds)
    pq = np.repeat(np.arange(ds.n_queries), ds.n_docs)
    pd = np.tile(np.arange(ds.n_docs), ds.n_queries)
    got, _ = check_pairs(ft, ds, ix, T, pq, pd, eps)
    if eps == 0.0:
        keys = ft.quadtree_pairs(ix, *queries(ds), t(pq), t(pd)).cpu().numpy().view(np.uint64)
        plain = keys.astype(np.float64) / float(1 << ds.Q)
        assert np.allclose(got, plain, rtol=1e-13, atol=0.0)


@pytest.mark.parametrize("case", ["dup_cluster", "grid28", "B8"])
def test_eps_pairs_small_cases(ft, case):
    X, shift, B = small_world(case)
    say("quadtree eps pairs:", case)
    ds = dataset_on(X, shift, B, 60, 4, 1, 25, 16, 21)
    ix = build_index(ft, ds)
    T = oracle_tree(ds)
    pq = np.repeat(np.arange(ds.n_queries), ds.n_docs)
    pd = np.tile(np.arange(ds.n_docs), ds.n_queries)
    for eps in (0.0, 0.3, 1.0):
        check_pairs(ft, ds, ix, T, pq, pd, eps)


def test_eps_pairs_text_shaped(ft):
    say("quadtree eps pairs: text-shaped V=20000 d=300, sizes to 500")
    ds = gen.make("text", V=20000, n_docs=120, n_queries=3)
    ix = build_index(ft, ds)
    T = oracle_tree(ds)
    pq = np.repeat(np.arange(ds.n_queries), ds.n_docs)
    pd = np.tile(np.arange(ds.n_docs), ds.n_queries)
    check_pairs(ft, ds, ix, T, pq, pd, 0.2)


def test_eps_identical_and_single_points(ft):
    """mu = nu gives 0; two point masses give the path weight between the two
    leaves, which is the same value the oracle reports for them."""
    say("quadtree eps pairs: identical distributions and point masses")
    ds = gen.make("tiny")
    ix = build_index(ft, ds)
    T = oracle_tree(ds)
    # queries: copies of docs 0..4, then five point masses
    ids = [ds.doc_id[ds.doc_off[d]:ds.doc_off[d + 1]] for d in range(5)]
    ms = [ds.doc_mass[ds.doc_off[d]:ds.doc_off[d + 1]] for d in range(5)]
    rng = np.random.default_rng(9)
    for p in rng.choice(ds.V, 5, replace=False):
        ids.append(np.array([p], np.uint32))
        ms.append(np.array([1 << ds.Q], np.uint32))
    off = np.zeros(len(ids) + 1, np.int64)
    off[1:] = np.cumsum([len(a) for a in ids])
    qi = np.concatenate(ids).astype(np.uint32)
    qm = np.concatenate(ms).astype(np.uint32)
    q = gen.Dataset("custom", ds.X, ds.shift, ds.B, ds.Q, ds.doc_off, ds.doc_id, ds.doc_mass, off, qi, qm, 5)
    eps = 0.3
    got = ft.quadtree_eps_pairs(ix, t(off), t(qi), t(qm), t(np.arange(5)), t(np.arange(5)), eps).cpu().numpy()
    assert np.abs(got).max() <= REL_SCALE * value_scale(ds.B, eps)
    pq = np.repeat(np.arange(5, 10), 5)
    pd = np.concatenate([np.arange(5)] * 5)
    check_pairs(ft, q, ix, T, pq, pd, eps)


@pytest.mark.parametrize("eps", [0.0, 0.35])
def test_eps_knn_candidates(ft, eps):
    say("quadtree eps knn: tiny, candidate lists, eps %.2f" % eps)
    ds = gen.make("tiny")
    ix = build_index(ft, ds)
    T = oracle_tree(ds)
    rng = np.random.default_rng(4)
    cand = np.stack([rng.choice(ds.n_docs, 300, replace=False) for _ in range(ds.n_queries)])
    cost, docs = ft.quadtree_eps_knn(ix, *queries(ds), 11, t(cand), eps)
    cost, docs = cost.cpu().numpy(), docs.cpu().numpy()
    swaps = 0
    for q in range(ds.n_queries):
        want = oracle_pairs(T, ds, np.full(cand.shape[1], q), cand[q], eps)
        swaps += check_topk(docs[q], cost[q], want, cand[q], 11)
    say("near-tie swaps:", swaps)


def test_eps_knn_grid_ties(ft):
    """Pixel grid: many candidates share a value; the order must still be
    (value, doc index) up to fp32 near-ties."""
    X, shift, B = small_world("grid28")
    say("quadtree eps knn: grid28, candidates with equal values")
    ds = dataset_on(X, shift, B, 400, 3, 1, 6, 16, 33)
    ix = build_index(ft, ds)
    T = oracle_tree(ds)
    cand = np.stack([np.arange(ds.n_docs)] * ds.n_queries)
    cost, docs = ft.quadtree_eps_knn(ix, *queries(ds), 25, t(cand), 0.5)
    cost, docs = cost.cpu().numpy(), docs.cpu().numpy()
    for q in range(ds.n_queries):
        want = oracle_pairs(T, ds, np.full(ds.n_docs, q), cand[q], 0.5)
        check_topk(docs[q], cost[q], want, cand[q], 25)


def test_eps_errors(ft):
    say("quadtree eps: error paths")
    ds = gen.make("tiny")
    ix = build_index(ft, ds)
    qo, qi, qm = queries(ds)
    one = t(np.zeros(1, np.int64))
    with pytest.raises(ft.FtError) as e:
        ft.quadtree_eps_pairs(ix, qo, qi, qm, one, one, -0.1)
    assert e.value.status == -1
    with pytest.raises(ft.FtError) as e:
        ft.quadtree_eps_pairs(ix, qo, qi, qm, one, one, 1.5)
    assert e.value.status == -1
    with pytest.raises(ft.FtError) as e:
        ft.quadtree_eps_pairs(ix, qo, qi, qm, one, t(np.array([ds.n_docs], np.int64)), 0.5)
    assert e.value.status == -1
    cand = t(np.zeros((ds.n_queries, 4097), np.int64))
    with pytest.raises(ft.FtError) as e:
        ft.quadtree_eps_knn(ix, qo, qi, qm, 3, cand, 0.5)
    assert e.value.status == -4
    # 500 pairs of coincident points: each pair hangs below a chain of cells
    # down to depth B, so a query over all 1000 points touches > 4096 cells
    rng = np.random.default_rng(12)
    X = np.repeat(rng.standard_normal((500, 2)).astype(np.float32), 2, axis=0)
    big = dataset_on(X, gen.random_shift(rng, 2, 30), 30, 3, 1, 1, 5, 24, 3)
    T = oracle_tree(big)
    assert T.n_nodes - 1 > 4096
    bix = build_index(ft, big)
    ids = np.arange(len(X), dtype=np.uint32)
    o = np.array([0, len(X)], np.int64)
    m = gen.uniform_masses(o, ids, big.Q)
    with pytest.raises(ft.FtError) as e:
        ft.quadtree_eps_pairs(bix, t(o), t(ids), t(m), one, one, 0.5)
    assert e.value.status == -4
    # the index still works afterwards
    got = ft.quadtree_eps_pairs(ix, qo, qi, qm, one, one, 0.5).cpu().numpy()
    assert np.isfinite(got).all()
