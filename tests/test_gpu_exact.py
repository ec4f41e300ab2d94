"""GPU parity of the exact W1 stage (ft_exact_pairs, ft_exact_knn) against
the oracle's exact solvers (Section 1, eq. (1)): successive shortest paths
in C for small pairs, the LP (HiGHS) for larger ones; every value within
1e-5 relative, top-k in the oracle's order up to near-ties.  Also the order
the paper's estimates must respect on the same pairs: ACT-1 <= W1 <= Flowtree
(GPU values)."""
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


def oracle_w1(ds, qo, qi, qm, pq, pd, solver):
    out = np.empty(len(pq))
    for p, (q, d) in enumerate(zip(pq, pd)):
        a, b = ds.doc_off[d], ds.doc_off[d + 1]
        qa, qb = qo[q], qo[q + 1]
        args = (ds.X, ds.doc_id[a:b], ds.doc_mass[a:b], qi[qa:qb], qm[qa:qb], ds.Q)
        out[p] = oracle.exact_w1_ssp(*args) if solver == "ssp" else oracle.exact_w1_lp(*args)
    return out


def check_values(got, want, what):
    got = np.asarray(got, np.float64)
    bad = np.abs(got - want) > RTOL_COST * np.abs(want) + 1e-30
    assert not bad.any(), "%s: %d of %d values off, first at %d: gpu %r oracle %r" % (
        what, bad.sum(), len(want), np.argmax(bad), got[np.argmax(bad)], want[np.argmax(bad)])


def test_exact_pairs_tiny(ft):
    say("exact W1 pairs: tiny workload (R^16), 10 queries x 40 docs, successive shortest paths oracle")
    ds = gen.make("tiny")
    ix = build_index(ft, ds)
    pq = np.repeat(np.arange(10), 40)
    pd = np.tile(np.arange(0, 500, 12)[:40], 10)
    got = ft.exact_pairs(ix, *queries(ds), t(pq), t(pd)).cpu().numpy()
    check_values(got, oracle_w1(ds, ds.q_off, ds.q_id, ds.q_mass, pq, pd, "ssp"), "exact W1")
    # the estimates bracket it on the same pairs
    act = ft.act_pairs(ix, *queries(ds), t(pq), t(pd), 1).cpu().numpy()
    assert (act <= got * (1 + 2e-5)).all()
    sel = np.arange(0, len(pq), 7)
    flow = [oracle.Tree(ds.X, ds.shift, ds.B).flowtree(
        ds.doc_id[ds.doc_off[d]:ds.doc_off[d + 1]], ds.doc_mass[ds.doc_off[d]:ds.doc_off[d + 1]],
        ds.q_id[ds.q_off[q]:ds.q_off[q + 1]], ds.q_mass[ds.q_off[q]:ds.q_off[q + 1]], Q=ds.Q)[0]
        for q, d in zip(pq[sel], pd[sel])]
    assert (got[sel] <= np.array(flow) * (1 + 2e-5)).all()


def test_exact_pairs_sizes(ft):
    """Text-shaped rows (R^300); queries on both sides of block edges
    against docs of up to 80 points, LP oracle."""
    say("exact W1 pairs: R^300, queries of 1..129 points, docs up to 80 points, LP oracle")
    ds = gen.make("text", V=4000, n_docs=200, n_queries=1, lo=1, hi=80)
    rng = np.random.default_rng(17)
    qsizes = [1, 2, 31, 33, 64, 129]
    qo, qi, qm = csr(rng, qsizes, ds.V, ds.Q)
    ix = build_index(ft, ds)
    sizes = np.diff(ds.doc_off)
    docs = np.concatenate([np.argsort(sizes)[-2:], rng.choice(ds.n_docs, 3, replace=False),
                           np.flatnonzero(sizes == 1)[:1]])
    pq = np.repeat(np.arange(len(qsizes)), len(docs))
    pd = np.tile(docs, len(qsizes))
    got = ft.exact_pairs(ix, t(qo), t(qi), t(qm), t(pq), t(pd)).cpu().numpy()
    check_values(got, oracle_w1(ds, qo, qi, qm, pq, pd, "lp"), "exact W1")


def test_exact_pairs_large_support(ft):
    """Queries of 513 and 1024 points (past the 512-item LDS layout, so the
    1024-item one runs) against docs of up to 80 points, and a 512-point
    query on its own index (the 512-item layout at its edge); successive
    shortest paths oracle."""
    say("exact W1 pairs: queries of 512, 513 and 1024 points in R^300, docs up to 80 points")
    ds = gen.make("text", V=4000, n_docs=60, n_queries=1, lo=1, hi=80)
    rng = np.random.default_rng(23)
    sizes = np.diff(ds.doc_off)
    docs = np.concatenate([np.argsort(sizes)[-2:], rng.choice(ds.n_docs, 2, replace=False)])
    for qsizes in ([512], [513, 1024]):
        qo, qi, qm = csr(rng, qsizes, ds.V, ds.Q)
        ix = build_index(ft, ds)
        pq = np.repeat(np.arange(len(qsizes)), len(docs))
        pd = np.tile(docs, len(qsizes))
        got = ft.exact_pairs(ix, t(qo), t(qi), t(qm), t(pq), t(pd)).cpu().numpy()
        check_values(got, oracle_w1(ds, qo, qi, qm, pq, pd, "ssp"), "exact W1, queries of %s points" % qsizes)


def test_exact_pairs_grid_ties(ft):
    say("exact W1 pairs: 28x28 grid, stroke images of 20..60 pixels (many equal costs)")
    ds = gen.make("image", n_docs=100, n_queries=4, lo=20, hi=60)
    ix = build_index(ft, ds)
    pq = np.repeat(np.arange(4), 10)
    pd = np.tile(np.arange(0, 100, 10), 4)
    got = ft.exact_pairs(ix, *queries(ds), t(pq), t(pd)).cpu().numpy()
    check_values(got, oracle_w1(ds, ds.q_off, ds.q_id, ds.q_mass, pq, pd, "lp"), "grid exact W1")


def test_exact_degenerate(ft):
    """Identical distributions: 0; single points: their distance."""
    say("exact W1 pairs: identical distributions and single points")
    ds = gen.make("tiny", n_docs=60, n_queries=2)
    qo = np.concatenate([ds.doc_off[:6], [ds.doc_off[5] + 1]])
    qi = np.concatenate([ds.doc_id[:ds.doc_off[5]], [7]]).astype(np.uint32)
    qm = np.concatenate([ds.doc_mass[:ds.doc_off[5]], [1 << ds.Q]]).astype(np.uint32)
    ix = build_index(ft, ds)
    got = ft.exact_pairs(ix, t(qo), t(qi), t(qm), t(np.arange(5)), t(np.arange(5))).cpu().numpy()
    assert (got == 0).all(), got
    one = np.flatnonzero(np.diff(ds.doc_off) >= 1)[:4]
    got = ft.exact_pairs(ix, t(qo), t(qi), t(qm), t(np.full(4, 5)), t(one)).cpu().numpy()
    check_values(got, oracle_w1(ds, qo, qi, qm, np.full(4, 5), one, "ssp"), "point mass")


def test_exact_knn_candidates(ft):
    say("exact W1 knn: tiny workload, 10 queries x 30 candidates")
    ds = gen.make("tiny")
    ix = build_index(ft, ds)
    rng = np.random.default_rng(5)
    cand = np.stack([rng.choice(ds.n_docs, 30, replace=False) for _ in range(ds.n_queries)]).astype(np.int64)
    costs, docs = ft.exact_knn(ix, *queries(ds), 30, cand=t(cand))
    c5, d5 = ft.exact_knn(ix, *queries(ds), 5, cand=t(cand))
    costs, docs, c5, d5 = [v.cpu().numpy() for v in (costs, docs, c5, d5)]
    for q in range(ds.n_queries):
        want = oracle_w1(ds, ds.q_off, ds.q_id, ds.q_mass, np.full(30, q), cand[q], "ssp")
        check_topk(docs[q], costs[q], want, cand[q], 30)
        check_topk(d5[q], c5[q], want, cand[q], 5)
