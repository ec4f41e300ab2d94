"""GPU parity of the Sinkhorn-k stage (ft_sinkhorn_pairs, ft_sinkhorn_knn)
against the float64 oracle (Section 4.1 baseline, regularisation from the
pair's largest cost with eta = 30): every value of explicit pairs within
1e-5 relative, and the top-k of candidate lists in the oracle's order up to
near-ties.  Sizes span several 32 x 32 blocks with ragged tails and queries
up to the largest support."""
import sys

import numpy as np
import pytest

import gen
import oracle
from gpu_util import RTOL_COST, build_index, check_topk, queries, t

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


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


def csr(rng, sizes, V, Q):
    sizes = np.asarray(sizes, np.int64)
    off, ids = gen.zipf_distinct(rng, sizes, V)
    return off, ids, gen.uniform_masses(off, ids, Q)


def oracle_pairs(ds, qo, qi, qm, pq, pd, iters, eta=30.0):
    return oracle.sinkhorn_pairs(ds.X, qo, qi, qm, ds.doc_off, ds.doc_id, ds.doc_mass, pq, pd, ds.Q, iters, eta)


def check_values(got, want, what):
    got = np.asarray(got, np.float64)
    bad = np.abs(got - want) > RTOL_COST * np.abs(want) + 1e-30
    assert not bad.any(), "%s: %d of %d values off, first at %d: gpu %r oracle %r" % (
        what, bad.sum(), len(want), np.argmax(bad), got[np.argmax(bad)], want[np.argmax(bad)])


@pytest.mark.parametrize("iters", [1, 3, 10])
def test_sinkhorn_pairs_tiny(ft, iters):
    say("Sinkhorn-%d pairs: tiny workload (R^16), 10 queries x 100 docs" % iters)
    ds = gen.make("tiny")
    ix = build_index(ft, ds)
    pq = np.repeat(np.arange(10), 100)
    pd = np.tile(np.arange(0, 500, 5), 10)
    got = ft.sinkhorn_pairs(ix, *queries(ds), t(pq), t(pd), iters).cpu().numpy()
    check_values(got, oracle_pairs(ds, ds.q_off, ds.q_id, ds.q_mass, pq, pd, iters), "Sinkhorn-%d" % iters)


@pytest.mark.parametrize("iters", [1, 3])
def test_sinkhorn_pairs_blocks(ft, iters):
    """Text-shaped rows (R^300); docs of 1..150 points, queries of sizes on
    both sides of every block edge, up to the largest support."""
    say("Sinkhorn-%d pairs: R^300, docs 1..150 points, queries up to 1024 points" % iters)
    ds = gen.make("text", V=4000, n_docs=300, n_queries=1, lo=1, hi=150)
    rng = np.random.default_rng(13)
    qsizes = [1, 2, 31, 32, 33, 64, 129, 300, 513, 1024]
    qo, qi, qm = csr(rng, qsizes, ds.V, ds.Q)
    ix = build_index(ft, ds)
    sizes = np.diff(ds.doc_off)
    docs = np.concatenate([np.argsort(sizes)[-4:], rng.choice(ds.n_docs, 8, replace=False),
                           np.flatnonzero(sizes == 1)[:2], np.flatnonzero(sizes == 33)[:1]])
    pq = np.repeat(np.arange(len(qsizes)), len(docs))
    pd = np.tile(docs, len(qsizes))
    got = ft.sinkhorn_pairs(ix, t(qo), t(qi), t(qm), t(pq), t(pd), iters).cpu().numpy()
    check_values(got, oracle_pairs(ds, qo, qi, qm, pq, pd, iters), "Sinkhorn-%d" % iters)


def test_sinkhorn_pairs_grid_and_eta(ft):
    """Image rows (28 x 28 grid in R^2, exact distance ties) and other
    regularisations."""
    say("Sinkhorn pairs: 28x28 grid, stroke images of 20..120 pixels, eta 30 / 5 / 100")
    ds = gen.make("image", n_docs=200, n_queries=6, lo=20, hi=120)
    ix = build_index(ft, ds)
    pq = np.repeat(np.arange(6), 40)
    pd = np.tile(np.arange(0, 200, 5), 6)
    for iters, eta in ((1, 30.0), (3, 5.0), (3, 100.0)):
        got = ft.sinkhorn_pairs(ix, *queries(ds), t(pq), t(pd), iters, eta).cpu().numpy()
        check_values(got, oracle_pairs(ds, ds.q_off, ds.q_id, ds.q_mass, pq, pd, iters, eta),
                     "grid Sinkhorn-%d eta %g" % (iters, eta))


def test_sinkhorn_point_masses(ft):
    """A side with one point: the estimate is the exact W1 (the product
    coupling); two single points give their distance; a pair of one shared
    point gives 0."""
    say("Sinkhorn pairs: point masses")
    rng = np.random.default_rng(4)
    X = gen.gaussian_mixture(rng, 200, 12, 3, 0.3, False)
    Q = 20
    doc_off, doc_id, doc_m = csr(rng, [1, 1, 9, 40], 200, Q)
    q_off, q_id, q_m = csr(rng, [1, 7, 1], 200, Q)
    q_id[0] = doc_id[0]  # query 0 is doc 0's point
    ds = gen.Dataset("points", X, gen.random_shift(rng, 12, 30), 30, Q, doc_off, doc_id, doc_m, q_off, q_id, q_m, 1)
    ix = build_index(ft, ds)
    pq = np.array([0, 2, 1, 2, 0, 0])
    pd = np.array([0, 1, 1, 2, 3, 2])
    for iters in (1, 3):
        got = ft.sinkhorn_pairs(ix, t(q_off), t(q_id), t(q_m), t(pq), t(pd), iters).cpu().numpy()
        want = oracle_pairs(ds, q_off, q_id, q_m, pq, pd, iters)
        assert got[0] == 0.0
        check_values(got[1:], want[1:], "point masses")
        D = lambda a, b: float(np.linalg.norm(X[a].astype(np.float64) - X[b]))
        assert abs(got[1] - D(q_id[q_off[2]], doc_id[doc_off[1]])) <= 1e-6 * got[1]


@pytest.mark.parametrize("iters", [1, 3])
def test_sinkhorn_knn_candidates(ft, iters):
    say("Sinkhorn-%d knn: text-shaped, 8 queries x 160 candidates" % iters)
    ds = gen.make("text", V=4000, n_docs=2000, n_queries=8, lo=5, hi=160)
    ix = build_index(ft, ds)
    rng = np.random.default_rng(3)
    cand = np.stack([rng.choice(ds.n_docs, 160, replace=False) for _ in range(ds.n_queries)]).astype(np.int64)
    costs, docs = ft.sinkhorn_knn(ix, *queries(ds), 160, iters=iters, cand=t(cand))
    c5, d5 = ft.sinkhorn_knn(ix, *queries(ds), 5, iters=iters, cand=t(cand))
    costs, docs, c5, d5 = [v.cpu().numpy() for v in (costs, docs, c5, d5)]
    swaps = 0
    for q in range(ds.n_queries):
        want = oracle_pairs(ds, ds.q_off, ds.q_id, ds.q_mass, np.full(160, q), cand[q], iters)
        swaps += check_topk(docs[q], costs[q], want, cand[q], 160)
        check_topk(d5[q], c5[q], want, cand[q], 5)
        assert (docs[q][:5] == d5[q]).all() and (costs[q][:5] == c5[q]).all()
    assert swaps <= 4


def test_sinkhorn_errors(ft):
    say("Sinkhorn: argument errors")
    ds = gen.make("tiny")
    ix = build_index(ft, ds)
    z = t(np.zeros(1, np.int64))
    for iters, eta in ((0, 30.0), (65, 30.0), (1, 0.0), (1, -1.0)):
        with pytest.raises(ft.FtError) as e:
            ft.sinkhorn_pairs(ix, *queries(ds), z, z, iters, eta)
        assert e.value.status == -1
    got = ft.sinkhorn_pairs(ix, *queries(ds), z, z, 2).cpu().numpy()
    check_values(got, oracle_pairs(ds, ds.q_off, ds.q_id, ds.q_mass, [0], [0], 2), "after errors")
