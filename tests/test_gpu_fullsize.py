"""The workloads at their full sizes, run the way bench.py runs them (all
queries in one call, Quadtree prune over every doc, batched Flowtree rerank),
checked against the CPU oracle on sampled queries and pairs: the exact
Quadtree top-k over every doc, the Flowtree top-k of the candidates, and
bit-exact flows for pairs from every size class.
"""
import sys

import numpy as np
import pytest

import gen
import oracle
from gpu_util import build_index, check_topk, oracle_flow_set, oracle_matrix, oracle_tree, queries, t

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


def pipeline_check(ft, ds, prune, k, sample, n_flow_pairs=120):
    """Prune all queries over all docs, rerank the candidates (batched), and
    check the sampled queries against the oracle; the one-call pipeline must
    give the same output bit for bit."""
    ix = build_index(ft, ds)
    qo, qi, qm = queries(ds)
    keys, cand = ft.quadtree_knn(ix, qo, qi, qm, prune)
    costs, docs = ft.flowtree_knn(ix, qo, qi, qm, k, cand=cand, mode=ft.FT_BATCHED)
    say("  the same search in one knn_pipeline call")
    p_costs, p_docs = ft.knn_pipeline(ix, qo, qi, qm, prune, k)
    torch.cuda.synchronize()
    assert torch.equal(p_docs, docs)
    assert torch.equal(p_costs.view(torch.int32), costs.view(torch.int32))
    keys, cand = keys.cpu().numpy().view(np.uint64), cand.cpu().numpy()
    costs, docs = costs.cpu().numpy(), docs.cpu().numpy()
    T = oracle_tree(ds)
    all_docs = np.arange(ds.n_docs)
    swaps = 0
    for q in sample:
        say("  query %d: oracle Quadtree over %d docs" % (q, ds.n_docs))
        M = oracle_matrix(T, ds, [q], all_docs, "qt")[0]
        check_topk(cand[q], keys[q], M, all_docs, prune, exact=True)
        F = oracle_matrix(T, ds, [q], cand[q], "ft")[0]
        swaps += check_topk(docs[q], costs[q], F, cand[q], k)
    # flows of sampled candidate pairs, the largest ones included
    rng = np.random.default_rng(7)
    sizes = np.diff(ds.doc_off)
    pairs = []
    for q in sample:
        c = cand[q]
        big = c[np.argsort(sizes[c])[-8:]]
        pairs += [(int(q), int(d)) for d in big]
        pairs += [(int(q), int(d)) for d in rng.choice(c, n_flow_pairs // len(sample), replace=False)]
    pq = np.array([p[0] for p in pairs])
    pd = np.array([p[1] for p in pairs])
    got = ft.flowtree_flows(ix, qo, qi, qm, t(pq), t(pd))
    for (q, d), (fd, fq, fe, fb) in zip(pairs, got):
        mine = sorted(zip(fd.tolist(), fq.tolist(), fe.tolist(), fb.tolist()))
        assert mine == oracle_flow_set(T, ds, q, d), "flow of pair (q=%d, doc=%d) differs" % (q, d)
    return swaps


def test_text_full(ft):
    say("full size: text-shaped, 100k docs, 1000 queries, prune 1000, rerank top-20")
    ds = gen.make("text")
    swaps = pipeline_check(ft, ds, 1000, 20, sample=[0, 517, 999])
    assert swaps <= 2


def test_batched_full(ft):
    say("full size: batched uneven, 1M docs, 4096 queries, prune 1000, rerank top-20")
    ds = gen.make("batched")
    swaps = pipeline_check(ft, ds, 1000, 20, sample=[0, 1500, 3999])
    assert swaps <= 2


def test_batched_prune_chunks(ft):
    """The 4096 queries of the batched workload twice over rank all 1M docs
    in four chunks of 2048 queries: two key buffers in turn, each one's key
    ranges cleared again by the select stream before its next chunk.  Both
    copies of every query must get the same top-1000 keys and docs, and a
    query of the last chunk must match the oracle's exact Quadtree top-k."""
    say("full size: 1M docs, the 4096 batched queries twice (four prune chunks), top-1000")
    ds = gen.make("batched")
    ix = build_index(ft, ds)
    nq = ds.n_queries
    off2 = np.concatenate([ds.q_off, ds.q_off[1:] + ds.q_off[-1]]).astype(np.int64)
    keys, cand = ft.quadtree_knn(ix, t(off2), t(np.tile(ds.q_id, 2)), t(np.tile(ds.q_mass, 2)), 1000)
    torch.cuda.synchronize()
    keys, cand = keys.cpu().numpy().view(np.uint64), cand.cpu().numpy()
    assert keys.shape == (2 * nq, 1000)
    assert np.array_equal(keys[:nq], keys[nq:])
    assert np.array_equal(cand[:nq], cand[nq:])
    q = nq - 5  # in the fourth chunk as query 2 * nq - 5
    say("  query %d: oracle Quadtree over %d docs" % (q, ds.n_docs))
    T = oracle_tree(ds)
    all_docs = np.arange(ds.n_docs)
    M = oracle_matrix(T, ds, [q], all_docs, "qt")[0]
    check_topk(cand[nq + q], keys[nq + q], M, all_docs, 1000, exact=True)


def test_image_full(ft):
    say("full size: image-shaped, 60k docs, 1000 queries, Flowtree over all docs, top-10")
    ds = gen.make("image")
    ix = build_index(ft, ds)
    qo, qi, qm = queries(ds)
    costs, docs = ft.flowtree_knn(ix, qo, qi, qm, 10, mode=ft.FT_BATCHED)
    keys, kd = ft.quadtree_knn(ix, qo, qi, qm, 10)
    costs, docs = costs.cpu().numpy(), docs.cpu().numpy()
    keys, kd = keys.cpu().numpy().view(np.uint64), kd.cpu().numpy()
    T = oracle_tree(ds)
    all_docs = np.arange(ds.n_docs)
    swaps = 0
    for q in (3, 640):
        say("  query %d: oracle Flowtree and Quadtree over %d docs" % (q, ds.n_docs))
        F = oracle_matrix(T, ds, [q], all_docs, "ft")[0]
        swaps += check_topk(docs[q], costs[q], F, all_docs, 10)
        M = oracle_matrix(T, ds, [q], all_docs, "qt")[0]
        check_topk(kd[q], keys[q], M, all_docs, 10, exact=True)
    assert swaps <= 2


def test_grad_full(ft):
    say("full size: gradient, V=50k d=300, 256 pairs, forward and backward")
    ds = gen.make("grad")
    ix = build_index(ft, ds)
    T = oracle_tree(ds)
    pq, pd = ds.extra["pair_q"], ds.extra["pair_d"]
    X = t(ds.X)
    qo, qi, qm = queries(ds)
    cost = torch.empty(len(pq), dtype=torch.float32, device=X.device)
    ft.flowtree_cost_grad(ix, X, qo, qi, qm, t(pq), t(pd), ft.FT_FWD, cost=cost)
    g_out = torch.linspace(0.25, 2.0, len(pq), device=X.device, dtype=torch.float32)
    gX = torch.zeros_like(X)
    gq = torch.zeros(len(ds.q_id), device=X.device)
    gd = torch.zeros(len(ds.doc_id), device=X.device)
    ft.flowtree_cost_grad(ix, X, qo, qi, qm, t(pq), t(pd), ft.FT_BWD, grad_out=g_out, grad_X=gX,
                          grad_qmass=gq, grad_dmass=gd)
    cost, gX, gq, gd, g_out = [v.cpu().numpy() for v in (cost, gX, gq, gd, g_out)]
    wX = {}
    wq = np.zeros(len(ds.q_id))
    wd = np.zeros(len(ds.doc_id))
    for p, (q, doc) in enumerate(zip(pq, pd)):
        a, b = ds.doc_off[doc], ds.doc_off[doc + 1]
        qa, qb = ds.q_off[q], ds.q_off[q + 1]
        mu, nu = ds.doc_id[a:b], ds.q_id[qa:qb]
        c, fl = T.flowtree(mu, ds.doc_mass[a:b], nu, ds.q_mass[qa:qb], Q=ds.Q)
        assert abs(cost[p] - c) <= 1e-5 * c
        # the frozen gradient on the pair's own rows
        rows = np.union1d(mu, nu)
        sub = ds.X[rows]
        gx, gm, gn = oracle.frozen_grad(sub, np.searchsorted(rows, mu), np.searchsorted(rows, nu), fl,
                                        ds.doc_mass[a:b] / 2.0 ** ds.Q, ds.q_mass[qa:qb] / 2.0 ** ds.Q)
        for i, r in enumerate(rows):
            wX[r] = wX.get(r, 0.0) + g_out[p] * gx[i]
        wd[a:b] += g_out[p] * gm
        wq[qa:qb] += g_out[p] * gn
    touched = np.array(sorted(wX))
    for r in touched:
        w = wX[r]
        assert np.linalg.norm(gX[r] - w) <= 1e-5 * np.linalg.norm(w) + 1e-7, "grad_X row %d" % r
    rest = np.setdiff1d(np.arange(len(ds.X)), touched)
    assert np.abs(gX[rest]).max() == 0
    assert np.allclose(gq, wq, rtol=1e-5, atol=1e-6 * np.abs(wq).max())
    assert np.allclose(gd, wd, rtol=1e-5, atol=1e-6 * np.abs(wd).max())
