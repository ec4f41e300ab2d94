"""GPU parity of the R-WMD / ACT-i stage (ft_act_pairs, ft_act_knn) against
the float64 oracle (Section 1.1 Relaxed WMD, Section 4.1 ACT-i): every value
of explicit pairs within 1e-5 relative, and the top-k of candidate lists in
the oracle's order up to near-ties.  Sizes span several 32 x 32 tiles with
ragged tails in both directions and all three query classes (<= 128, <= 512,
<= 1024 points); the grid data of the image workload forces exact distance
ties."""
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
    """Distributions of the given support sizes over Zipf(1.1) distinct
    points of [0, V), uniform masses summing to 2^Q."""
    sizes = np.asarray(sizes, np.int64)
    off, ids = gen.zipf_distinct(rng, sizes, V)
    return off, ids, gen.uniform_masses(off, ids, Q)


def oracle_pairs(ds, qo, qi, qm, pq, pd, iters):
    return oracle.act_pairs(ds.X, qo, qi, qm, ds.doc_off, ds.doc_id, ds.doc_mass, pq, pd, ds.Q, iters)


def check_values(got, want, what):
    got = np.asarray(got, np.float64)
    bad = np.abs(got - want) > RTOL_COST * np.abs(want) + 1e-30
    assert not bad.any(), "%s: %d of %d values off, first at %d: gpu %r oracle %r" % (
        what, bad.sum(), len(want), np.argmax(bad), got[np.argmax(bad)], want[np.argmax(bad)])


@pytest.mark.parametrize("iters", [0, 1, 2, 3, 7])
def test_act_pairs_tiny(ft, iters):
    say("ACT-%d pairs: tiny workload (R^16), 10 queries x 100 docs" % iters)
    ds = gen.make("tiny")
    ix = build_index(ft, ds)
    pq = np.repeat(np.arange(10), 100)
    pd = np.tile(np.arange(0, 500, 5), 10)
    got = ft.act_pairs(ix, *queries(ds), t(pq), t(pd), iters).cpu().numpy()
    want = oracle_pairs(ds, ds.q_off, ds.q_id, ds.q_mass, pq, pd, iters)
    check_values(got, want, "ACT-%d" % iters)
    if iters == 0:
        r = np.array([oracle.rwmd(ds.X, ds.doc_id[ds.doc_off[d]:ds.doc_off[d + 1]],
                                  ds.doc_mass[ds.doc_off[d]:ds.doc_off[d + 1]],
                                  ds.q_id[ds.q_off[q]:ds.q_off[q + 1]], ds.q_mass[ds.q_off[q]:ds.q_off[q + 1]], ds.Q)
                      for q, d in zip(pq, pd)])
        check_values(got, r, "R-WMD")


@pytest.mark.parametrize("iters", [0, 1])
def test_act_pairs_tiles_and_classes(ft, iters):
    """Text-shaped rows (R^300, unit norm); docs of 1..150 points, queries of
    sizes on both sides of every tile edge and class edge."""
    say("ACT-%d pairs: R^300, docs 1..150 points, queries up to 1024 points" % iters)
    ds = gen.make("text", V=4000, n_docs=300, n_queries=1, lo=1, hi=150)
    rng = np.random.default_rng(11)
    qsizes = [1, 2, 31, 32, 33, 64, 127, 128, 129, 300, 511, 512, 513, 700, 1024]
    qo, qi, qm = csr(rng, qsizes, ds.V, ds.Q)
    ix = build_index(ft, ds)
    sizes = np.diff(ds.doc_off)
    docs = np.concatenate([np.argsort(sizes)[-6:], rng.choice(ds.n_docs, 10, replace=False),
                           np.flatnonzero(sizes == 1)[:2], np.flatnonzero(sizes == 32)[:1],
                           np.flatnonzero(sizes == 33)[:1]])
    pq = np.repeat(np.arange(len(qsizes)), len(docs))
    pd = np.tile(docs, len(qsizes))
    got = ft.act_pairs(ix, t(qo), t(qi), t(qm), t(pq), t(pd), iters).cpu().numpy()
    want = oracle_pairs(ds, qo, qi, qm, pq, pd, iters)
    check_values(got, want, "ACT-%d" % iters)


def test_act_pairs_grid_ties(ft):
    """Image workload rows (28 x 28 grid in R^2): many points of the other
    side at exactly the same distance."""
    say("ACT pairs: 28x28 grid, stroke images of 20..120 pixels")
    ds = gen.make("image", n_docs=200, n_queries=6, lo=20, hi=120)
    ix = build_index(ft, ds)
    pq = np.repeat(np.arange(6), 40)
    pd = np.tile(np.arange(0, 200, 5), 6)
    for iters in (0, 1, 4):
        got = ft.act_pairs(ix, *queries(ds), t(pq), t(pd), iters).cpu().numpy()
        want = oracle_pairs(ds, ds.q_off, ds.q_id, ds.q_mass, pq, pd, iters)
        check_values(got, want, "grid ACT-%d" % iters)


def test_act_degenerate(ft):
    """Identical distributions give 0; single points give the distance;
    coincident coordinates under different ids are at distance 0."""
    say("ACT pairs: degenerate cases")
    rng = np.random.default_rng(5)
    X = gen.gaussian_mixture(rng, 300, 24, 4, 0.3, False)
    X[200:220] = X[0:20]  # twenty coincident pairs of points
    Q = 20
    doc_off, doc_id, doc_m = csr(rng, [1, 5, 40, 70], 300, Q)
    doc_off = np.concatenate([doc_off, doc_off[-1] + np.array([20])])
    doc_id = np.concatenate([doc_id, np.arange(200, 220, dtype=np.uint32)])
    doc_m = np.concatenate([doc_m, gen.uniform_masses(np.array([0, 20]), np.arange(200, 220, dtype=np.uint32), Q)])
    ds = gen.Dataset("degenerate", X, gen.random_shift(rng, 24, 30), 30, Q, doc_off, doc_id, doc_m,
                     doc_off.copy(), doc_id.copy(), doc_m.copy(), 1)
    qo, qi, qm = ds.q_off, ds.q_id, ds.q_mass
    # the query set also holds the duplicate image of doc 4 (ids 0..19)
    qo = np.concatenate([qo, [qo[-1] + 20]])
    qi = np.concatenate([qi, np.arange(0, 20, dtype=np.uint32)])
    qm = np.concatenate([qm, doc_m[doc_off[4]:doc_off[5]]])
    ix = build_index(ft, ds)
    n = 5
    pq = np.concatenate([np.arange(n), np.repeat(np.arange(n + 1), n)])
    pd = np.concatenate([np.arange(n), np.tile(np.arange(n), n + 1)])
    for iters in (0, 1, 2):
        got = ft.act_pairs(ix, t(qo), t(qi), t(qm), t(pq), t(pd), iters).cpu().numpy()
        assert (got[:n] == 0).all(), got[:n]
        want = oracle_pairs(ds, qo, qi, qm, pq, pd, iters)
        check_values(got, want, "degenerate ACT-%d" % iters)
        assert got[n + 5 * n + 4] == 0.0  # ids 200..219 against their copies 0..19


@pytest.mark.parametrize("iters", [0, 1])
def test_act_knn_candidates(ft, iters):
    """Candidate lists per query (the pipeline form): the full ordered list
    (k = n_cand) and a top-5, against the oracle over the same candidates."""
    say("ACT-%d knn: text-shaped, 8 queries x 160 candidates" % iters)
    ds = gen.make("text", V=4000, n_docs=2000, n_queries=8, lo=5, hi=160)
    ix = build_index(ft, ds)
    rng = np.random.default_rng(3)
    cand = np.stack([rng.choice(ds.n_docs, 160, replace=False) for _ in range(ds.n_queries)]).astype(np.int64)
    costs, docs = ft.act_knn(ix, *queries(ds), 160, iters=iters, cand=t(cand))
    c5, d5 = ft.act_knn(ix, *queries(ds), 5, iters=iters, cand=t(cand))
    costs, docs, c5, d5 = [v.cpu().numpy() for v in (costs, docs, c5, d5)]
    swaps = 0
    for q in range(ds.n_queries):
        want = oracle_pairs(ds, ds.q_off, ds.q_id, ds.q_mass, np.full(160, q), cand[q], iters)
        swaps += check_topk(docs[q], costs[q], want, cand[q], 160)
        check_topk(d5[q], c5[q], want, cand[q], 5)
        assert (docs[q][:5] == d5[q]).all() and (costs[q][:5] == c5[q]).all()
    assert swaps <= 4


def test_act_errors(ft):
    say("ACT: argument errors")
    ds = gen.make("text", V=4000, n_docs=50, n_queries=1, lo=5, hi=50)
    ix = build_index(ft, ds)
    z = t(np.zeros(1, np.int64))
    with pytest.raises(ft.FtError) as e:
        ft.act_pairs(ix, *queries(ds), z, z, 8)
    assert e.value.status == -1
    rng = np.random.default_rng(2)
    qo, qi, qm = csr(rng, [2100], ds.V, ds.Q)
    with pytest.raises(ft.FtError) as e:
        ft.act_pairs(ix, t(qo), t(qi), t(qm), z, z, 1)
    assert e.value.status == -4
    # the index still works afterwards, with a largest query and 7 iterations
    qo, qi, qm = csr(rng, [1024], ds.V, ds.Q)
    got = ft.act_pairs(ix, t(qo), t(qi), t(qm), z, z, 7).cpu().numpy()
    want = oracle_pairs(ds, qo, qi, qm, [0], [0], 7)
    check_values(got, want, "after errors")
