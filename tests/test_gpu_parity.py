"""HIP path against the CPU oracle, through the C ABI.

Bars: bit-exact tree (Morton order, adjacent LCA depths, leaf depths), bit-
exact Quadtree keys and Flowtree flows; float32 Flowtree costs within 1e-5
relative of the float64 oracle; identical top-k (near-ties within 2e-5
relative may swap, and are counted).
"""
import sys

import numpy as np
import pytest

import gen
import oracle
from gpu_util import (build_index, check_topk, oracle_flow_set, oracle_matrix, oracle_tree,
                      queries, subset, t)

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


# ------------------------------------------------------------------ worlds --

def world_tiny():
    return gen.make("tiny")


def world_small_cases():
    """Hand-made ground sets stressing the tree: coincident points (depth-B
    leaves holding several points), tight clusters (deep trees), a grid."""
    out = []
    rng = np.random.default_rng(5)
    X = rng.standard_normal((300, 3)).astype(np.float32)
    X[100:110] = X[0]                       # ten coincident points
    X[200:260] = (X[200:260] * 1e-4 + 3).astype(np.float32)  # a tight cluster
    out.append(("dup_cluster", X, gen.random_shift(rng, 3, 30), 30))
    out.append(("grid28", gen.pixel_grid(28), gen.random_shift(rng, 2, 30), 30))
    out.append(("B8", rng.standard_normal((200, 2)).astype(np.float32), gen.random_shift(rng, 2, 8), 8))
    return out


def dataset_on(X, shift, B, n_docs, n_q, lo, hi, Q, seed):
    rng = np.random.default_rng(seed)
    V = len(X)
    def dists(n):
        sizes = rng.integers(lo, min(hi, V) + 1, size=n)
        off = np.zeros(n + 1, np.int64)
        off[1:] = np.cumsum(sizes)
        ids = np.concatenate([rng.choice(V, s, replace=False) for s in sizes]).astype(np.uint32)
        m = gen.uniform_masses(off, ids, Q)
        return off, ids, m
    do, di, dm = dists(n_docs)
    qo, qi, qm = dists(n_q)
    return gen.Dataset("custom", X, np.asarray(shift, np.int64), B, Q, do, di, dm, qo, qi, qm, 5)


# ------------------------------------------------------------------- tree --

def check_tree(ft, ds):
    ix = build_index(ft, ds)
    perm, lcp, ld = ix.export_tree()
    T = oracle_tree(ds)
    ex = T.export()
    point_at = np.argsort(ex["rank_of"])
    perm = perm.cpu().numpy().astype(np.int64)
    assert (perm == point_at).all(), "Morton order differs"
    lcp = lcp.cpu().numpy().astype(np.int64)
    want = [T.lca_depth(point_at[r], point_at[r + 1]) for r in range(len(perm) - 1)]
    assert (lcp[:-1] == np.array(want)).all(), "adjacent LCA depths differ"
    ld = ld.cpu().numpy().astype(np.int64)
    assert (ld == ex["leaf_depth"][point_at]).all(), "leaf depths differ"
    info = ix.info()
    assert info["n_nodes"] == T.n_nodes
    assert info["height"] == ex["leaf_depth"].max()
    return ix, T


def test_tree_tiny(ft):
    say("tree: tiny")
    check_tree(ft, world_tiny())


@pytest.mark.parametrize("case", range(3))
def test_tree_small_cases(ft, case):
    name, X, shift, B = world_small_cases()[case]
    say("tree:", name)
    ds = dataset_on(X, shift, B, 40, 4, 1, 20, 16, case)
    check_tree(ft, ds)


def test_tree_text_shaped(ft):
    say("tree: text-shaped V=20000 d=300")
    ds = gen.make("text", V=20000, n_docs=200, n_queries=2)
    check_tree(ft, ds)


# --------------------------------------------------------------- quadtree --

def test_quadtree_pairs_bitexact_tiny(ft):
    say("quadtree pairs: tiny, all 5000 pairs")
    ds = world_tiny()
    ix = build_index(ft, ds)
    T = oracle_tree(ds)
    pq = np.repeat(np.arange(ds.n_queries), ds.n_docs)
    pd = np.tile(np.arange(ds.n_docs), ds.n_queries)
    got = ft.quadtree_pairs(ix, *queries(ds), t(pq), t(pd)).cpu().numpy().view(np.uint64)
    want = T.quadtree_pairs(ds.q_off, ds.q_id, ds.q_mass, ds.doc_off, ds.doc_id, ds.doc_mass, pq, pd, ds.Q)
    assert (got == want).all()


@pytest.mark.parametrize("case", range(3))
def test_quadtree_knn_small_cases(ft, case):
    name, X, shift, B = world_small_cases()[case]
    say("quadtree knn:", name)
    ds = dataset_on(X, shift, B, 150, 5, 1, 25, 16, 10 + case)
    ix = build_index(ft, ds)
    T = oracle_tree(ds)
    keys, docs = ft.quadtree_knn(ix, *queries(ds), 7)
    keys = keys.cpu().numpy().view(np.uint64)
    docs = docs.cpu().numpy()
    M = oracle_matrix(T, ds, range(ds.n_queries), np.arange(ds.n_docs), "qt")
    for q in range(ds.n_queries):
        check_topk(docs[q], keys[q], M[q], np.arange(ds.n_docs), 7, exact=True)


def test_quadtree_knn_tiny_all_and_cand(ft):
    say("quadtree knn: tiny, all docs and candidate lists")
    ds = world_tiny()
    ix = build_index(ft, ds)
    T = oracle_tree(ds)
    M = oracle_matrix(T, ds, range(ds.n_queries), np.arange(ds.n_docs), "qt")
    keys, docs = ft.quadtree_knn(ix, *queries(ds), ds.k)
    for q in range(ds.n_queries):
        check_topk(docs[q].cpu().numpy(), keys[q].cpu().numpy().view(np.uint64), M[q], np.arange(ds.n_docs),
                   ds.k, exact=True)
    rng = np.random.default_rng(3)
    cand = np.stack([rng.choice(ds.n_docs, 77, replace=False) for _ in range(ds.n_queries)])
    keys, docs = ft.quadtree_knn(ix, *queries(ds), 9, cand=t(cand))
    for q in range(ds.n_queries):
        check_topk(docs[q].cpu().numpy(), keys[q].cpu().numpy().view(np.uint64), M[q][cand[q]], cand[q], 9,
                   exact=True)


@pytest.mark.parametrize("Q", [25, 30, 31])
def test_quadtree_knn_counter_modes(ft, Q):
    """Ranking all docs at the edges of its arithmetic modes (tiny set, tree
    height 7): Q + height = 32 keeps 32-bit counters but 64-bit keys; above
    32 the counters are 64-bit too (the usual Q = 24 case, height 7, packs
    keys into 32 bits and is covered elsewhere)."""
    say("quadtree knn: tiny with Q=%d" % Q)
    ds = gen.make("tiny", Q=Q, n_docs=1500, n_queries=6)
    ix = build_index(ft, ds)
    assert ix.info()["height"] == 7
    T = oracle_tree(ds)
    docs = np.arange(ds.n_docs)
    M = oracle_matrix(T, ds, range(ds.n_queries), docs, "qt")
    keys, kd = ft.quadtree_knn(ix, *queries(ds), 40)
    for q in range(ds.n_queries):
        check_topk(kd[q].cpu().numpy(), keys[q].cpu().numpy().view(np.uint64), M[q], docs, 40, exact=True)


# --------------------------------------------------------------- flowtree --

def check_flows(ft, ds, ix, T, pairs, q_sel=None):
    qc = None
    if q_sel is not None:
        qc = subset(ds.q_off, ds.q_id, ds.q_mass, q_sel)
    pq = np.array([p[0] for p in pairs])
    pd = np.array([p[1] for p in pairs])
    got = ft.flowtree_flows(ix, *(queries(ds) if qc is None else (t(qc[0]), t(qc[1]), t(qc[2]))),
                            t(pq), t(pd))
    for (q, doc), (fd, fq, fe, fb) in zip(pairs, got):
        mine = sorted(zip(fd.tolist(), fq.tolist(), fe.tolist(), fb.tolist()))
        want = oracle_flow_set(T, ds, q, doc, q_csr=qc)
        assert mine == want, "flow of pair (q=%d, doc=%d) differs" % (q, doc)


def test_flows_bitexact_tiny(ft):
    say("flows: tiny, 400 pairs")
    ds = world_tiny()
    ix = build_index(ft, ds)
    T = oracle_tree(ds)
    rng = np.random.default_rng(0)
    pairs = [(int(rng.integers(ds.n_queries)), int(rng.integers(ds.n_docs))) for _ in range(400)]
    check_flows(ft, ds, ix, T, pairs)


@pytest.mark.parametrize("case", range(3))
def test_flows_bitexact_small_cases(ft, case):
    name, X, shift, B = world_small_cases()[case]
    say("flows:", name)
    ds = dataset_on(X, shift, B, 60, 6, 1, 40, 12, 20 + case)
    ix = build_index(ft, ds)
    T = oracle_tree(ds)
    pairs = [(q, doc) for q in range(ds.n_queries) for doc in range(0, ds.n_docs, 3)]
    check_flows(ft, ds, ix, T, pairs)


def test_flows_shared_points(ft):
    """Queries equal to docs, and sharing most points: self-matches at leaves."""
    say("flows: shared supports")
    ds = world_tiny()
    sel = [0, 1, 2, 3]
    qo, qi, qm = subset(ds.doc_off, ds.doc_id, ds.doc_mass, sel)
    ds2 = gen.Dataset("shared", ds.X, ds.shift, ds.B, ds.Q, ds.doc_off, ds.doc_id, ds.doc_mass, qo, qi, qm, 5)
    ix = build_index(ft, ds2)
    T = oracle_tree(ds2)
    pairs = [(q, doc) for q in range(4) for doc in range(8)]
    check_flows(ft, ds2, ix, T, pairs)
    costs, docs = ft.flowtree_knn(ix, *queries(ds2), 3, mode=ft.FT_BATCHED)
    assert (docs[:, 0].cpu().numpy() == np.array(sel)).all()
    assert (costs[:, 0].cpu().numpy() == 0).all()


def test_flows_class_edges_and_max_support(ft):
    """Pairs of 2 to 2048 merged items: both sides of every size-class edge
    (128/129, 256/257, 512/513, 1024/1025), the largest supports (1024 +
    1024) and single-point distributions.  Flows bit-exact, costs to the
    oracle, plain == batched."""
    say("flows: size-class edges, single points, 1024 + 1024 items")
    base = gen.make("tiny", n_docs=2, n_queries=1)
    rng = np.random.default_rng(11)

    def csr(sizes):
        off = np.zeros(len(sizes) + 1, np.int64)
        off[1:] = np.cumsum(sizes)
        ids = np.concatenate([rng.choice(base.V, s, replace=False) for s in sizes]).astype(np.uint32)
        return off, ids, gen.uniform_masses(off, ids, base.Q)

    do, di, dm = csr([1, 63, 64, 65, 192, 193, 448, 449, 960, 961, 1024])
    qo, qi, qm = csr([1, 64, 1024])
    ds = gen.Dataset("edges", base.X, base.shift, base.B, base.Q, do, di, dm, qo, qi, qm, 5)
    ix = build_index(ft, ds)
    T = oracle_tree(ds)
    check_flows(ft, ds, ix, T, [(q, d) for q in range(3) for d in range(ds.n_docs)])
    flow_knn_check(ft, ds, ix, T, ds.n_docs)


def flow_knn_check(ft, ds, ix, T, k, cand=None, modes=("plain", "batched"), q_sel=None):
    n_q = ds.n_queries
    res = {}
    for mode in modes:
        m = ft.FT_PLAIN if mode == "plain" else ft.FT_BATCHED
        c, d = ft.flowtree_knn(ix, *queries(ds), k, cand=None if cand is None else t(cand), mode=m)
        res[mode] = (c.cpu().numpy(), d.cpu().numpy())
    if len(modes) == 2:
        assert (res["plain"][1] == res["batched"][1]).all()
        assert (res["plain"][0] == res["batched"][0]).all(), "plain and batched costs differ"
    c, d = res[modes[-1]]
    swaps = 0
    qs = range(n_q) if q_sel is None else q_sel
    for q in qs:
        cols = np.arange(ds.n_docs) if cand is None else cand[q]
        M = oracle_matrix(T, ds, [q], cols, "ft")[0]
        swaps += check_topk(d[q], c[q], M, cols, k)
    return swaps


def test_flowtree_knn_tiny_full_ranking(ft):
    say("flowtree knn: tiny, full ranking of 500 docs, plain and batched")
    ds = world_tiny()
    ix = build_index(ft, ds)
    T = oracle_tree(ds)
    swaps = flow_knn_check(ft, ds, ix, T, ds.n_docs)
    say("  near-tie swaps:", swaps)
    swaps = flow_knn_check(ft, ds, ix, T, ds.k)
    assert swaps == 0


def test_flowtree_knn_text_reduced_pipeline(ft):
    say("pipeline: text-shaped V=5000 d=300, 2000 docs, 6 queries: quadtree 100 -> flowtree 20")
    ds = gen.make("text", V=5000, n_docs=2000, n_queries=6)
    ix = build_index(ft, ds)
    T = oracle_tree(ds)
    keys, cand = ft.quadtree_knn(ix, *queries(ds), 100)
    M = oracle_matrix(T, ds, range(ds.n_queries), np.arange(ds.n_docs), "qt")
    cand_h = cand.cpu().numpy()
    for q in range(ds.n_queries):
        check_topk(cand_h[q], keys[q].cpu().numpy().view(np.uint64), M[q], np.arange(ds.n_docs), 100, exact=True)
    swaps = flow_knn_check(ft, ds, ix, T, 20, cand=cand_h)
    assert swaps == 0


def test_flowtree_knn_image_reduced(ft):
    say("flowtree knn: image-shaped, 1500 docs, 3 queries, all docs, top-10")
    ds = gen.make("image", n_docs=1500, n_queries=3)
    ix = build_index(ft, ds)
    T = oracle_tree(ds)
    flow_knn_check(ft, ds, ix, T, 10)


def test_flowtree_knn_uneven_sizes(ft):
    say("flowtree knn: sizes 5..500 (power law), V=4000 d=300, 1500 docs, 8 queries, all size classes")
    ds = gen.make("batched", V=4000, n_docs=1500, n_queries=8)
    # make sure the largest class is exercised
    assert np.diff(ds.q_off).max() + np.diff(ds.doc_off).max() > 512
    ix = build_index(ft, ds)
    T = oracle_tree(ds)
    rng = np.random.default_rng(1)
    cand = np.stack([rng.choice(ds.n_docs, 300, replace=False) for _ in range(ds.n_queries)])
    flow_knn_check(ft, ds, ix, T, 20, cand=cand)


def test_flowtree_deterministic(ft):
    say("flowtree knn: repeated batched calls give identical bits")
    ds = world_tiny()
    ix = build_index(ft, ds)
    a = ft.flowtree_knn(ix, *queries(ds), 50, mode=ft.FT_BATCHED)
    b = ft.flowtree_knn(ix, *queries(ds), 50, mode=ft.FT_BATCHED)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


# ------------------------------------------------------------- gradients --

def oracle_weighted_grad(ds, pq, pd, g_out):
    """Oracle Flowtree costs of the pairs and the float64 frozen gradient of
    sum_p g_out[p] cost_p in X, the query weights and the doc weights."""
    T = oracle_tree(ds)
    costs = np.empty(len(pq))
    wX = np.zeros(ds.X.shape)
    wq = np.zeros(len(ds.q_id))
    wd = np.zeros(len(ds.doc_id))
    for p, (q, doc) in enumerate(zip(pq, pd)):
        a, b = ds.doc_off[doc], ds.doc_off[doc + 1]
        qa, qb = ds.q_off[q], ds.q_off[q + 1]
        costs[p], fl = T.flowtree(ds.doc_id[a:b], ds.doc_mass[a:b], ds.q_id[qa:qb], ds.q_mass[qa:qb], Q=ds.Q)
        gx, gm, gn = oracle.frozen_grad(ds.X, ds.doc_id[a:b], ds.q_id[qa:qb], fl,
                                        ds.doc_mass[a:b] / 2.0 ** ds.Q, ds.q_mass[qa:qb] / 2.0 ** ds.Q)
        wX += g_out[p] * gx
        wd[a:b] += g_out[p] * gm
        wq[qa:qb] += g_out[p] * gn
    return costs, wX, wq, wd


def assert_grads_close(gX, gq, gd, wX, wq, wd):
    """1e-5 relative in norm per nonzero row of dX; rows the oracle leaves
    at zero stay exactly zero; weight gradients 1e-5 relative."""
    rows = np.flatnonzero(np.abs(wX).sum(1) > 0)
    for r in rows:
        assert np.linalg.norm(gX[r] - wX[r]) <= 1e-5 * np.linalg.norm(wX[r]) + 1e-7, "row %d" % r
    untouched = np.setdiff1d(np.arange(len(wX)), rows)
    assert (gX[untouched] == 0).all()
    assert np.allclose(gq, wq, rtol=1e-5, atol=1e-6 * np.abs(wq).max())
    assert np.allclose(gd, wd, rtol=1e-5, atol=1e-6 * np.abs(wd).max())


def check_cost_grad(ft, ds, pq, pd, g_lo, g_hi):
    """Forward costs and the backward (X, query weights, doc weights) of
    sum_p g_p cost_p against the oracle's Flowtree and its float64 frozen
    gradient."""
    ix = build_index(ft, ds)
    X = t(ds.X)
    qo, qi, qm = queries(ds)
    cost = torch.empty(len(pq), dtype=torch.float32, device=X.device)
    ft.flowtree_cost_grad(ix, X, qo, qi, qm, t(pq), t(pd), ft.FT_FWD, cost=cost)
    g_out = torch.linspace(g_lo, g_hi, len(pq), device=X.device, dtype=torch.float32)
    gX = torch.zeros_like(X)
    gq = torch.zeros(len(ds.q_id), device=X.device)
    gd = torch.zeros(len(ds.doc_id), device=X.device)
    ft.flowtree_cost_grad(ix, X, qo, qi, qm, t(pq), t(pd), ft.FT_BWD, grad_out=g_out, grad_X=gX,
                          grad_qmass=gq, grad_dmass=gd)
    cost, gX, gq, gd, g_out = [v.cpu().numpy() for v in (cost, gX, gq, gd, g_out)]
    want, wX, wq, wd = oracle_weighted_grad(ds, pq, pd, g_out)
    assert (np.abs(cost - want) <= 1e-5 * want).all()
    assert_grads_close(gX, gq, gd, wX, wq, wd)


def test_cost_grad_vs_oracle(ft):
    say("cost_grad: V=3000 d=300, 24 pairs, forward and backward")
    ds = gen.make("grad", V=3000, n_pairs=24)
    check_cost_grad(ft, ds, ds.extra["pair_q"], ds.extra["pair_d"], 0.5, 1.5)


@pytest.mark.parametrize("hi,d", [(60, 30), (120, 32), (250, 30), (500, 32), (1000, 30)])
def test_cost_grad_size_classes(ft, hi, d):
    """Forward and backward in every size class (the largest pair of a call
    picks the workgroup shape: up to 128, 256, 512, 1024 and 2048 items),
    with rows of d = 30 (scalar loads) and d = 32 (float4 loads); some
    queries share points with their docs, and one pair is a distribution
    against itself (every match a zero-length self-match)."""
    say("cost_grad size class: supports up to %d, d=%d" % (hi, d))
    rng = np.random.default_rng(900 + hi)
    X = rng.standard_normal((3000, d)).astype(np.float32)
    X[10:14] = X[5]  # coincident points under different ids
    ds = dataset_on(X, gen.random_shift(rng, d, 30), 30, 6, 4, max(1, hi // 3), hi, 24, hi)
    # query 0 is doc 0 itself; query 1 shares half of doc 1's points
    do, di, dm = ds.doc_off, ds.doc_id.copy(), ds.doc_mass
    qo, qi, qm = ds.q_off, ds.q_id.copy(), ds.q_mass
    n0 = do[1] - do[0]
    qsz = np.diff(qo)
    qsz[0] = n0
    nqo = np.zeros(len(qsz) + 1, np.int64)
    nqo[1:] = np.cumsum(qsz)
    nqi = np.concatenate([di[do[0]:do[1]]] + [qi[qo[j]:qo[j + 1]] for j in range(1, len(qsz))]).astype(np.uint32)
    a1, b1 = do[1], do[2]
    share = di[a1:a1 + (b1 - a1) // 2]
    q1 = nqi[nqo[1]:nqo[2]]
    keep = np.setdiff1d(q1, share)[: max(0, len(q1) - len(share))]
    q1 = np.concatenate([share, keep])[: len(q1)]
    assert len(np.unique(q1)) == len(q1)
    nqi[nqo[1]:nqo[2]] = q1
    nqm = gen.uniform_masses(nqo, nqi, 24)
    ds = gen.Dataset("custom", X, ds.shift, 30, 24, do, di, dm, nqo, nqi, nqm, 5)
    pq = np.array([0, 1, 2, 3, 0, 1, 2, 3, 3], np.int64)
    pd = np.array([0, 1, 2, 3, 4, 5, 5, 4, 0], np.int64)
    check_cost_grad(ft, ds, pq, pd, 0.25, 2.0)


def test_cost_grad_deterministic(ft):
    """Two backward calls over pairs that share queries and docs (so several
    pairs add into the same rows of dX and the same weights) give the same
    gradients to the bit, and they match the oracle; a non-finite grad_out
    is rejected."""
    say("cost_grad: bit-identical gradients across calls, shared rows")
    ds = gen.make("grad", V=3000, n_pairs=16)
    rng = np.random.default_rng(41)
    pq = rng.integers(0, 4, 64).astype(np.int64)
    pd = rng.integers(0, 6, 64).astype(np.int64)
    ix = build_index(ft, ds)
    X = t(ds.X)
    qo, qi, qm = queries(ds)
    cost = torch.empty(len(pq), dtype=torch.float32, device=X.device)
    ft.flowtree_cost_grad(ix, X, qo, qi, qm, t(pq), t(pd), ft.FT_FWD, cost=cost)
    g_out = torch.from_numpy(rng.uniform(-2.0, 3.0, len(pq)).astype(np.float32)).to(X.device)
    runs = []
    for _ in range(2):
        gX = torch.zeros_like(X)
        gq = torch.zeros(len(ds.q_id), device=X.device)
        gd = torch.zeros(len(ds.doc_id), device=X.device)
        ft.flowtree_cost_grad(ix, X, qo, qi, qm, t(pq), t(pd), ft.FT_BWD, grad_out=g_out, grad_X=gX,
                              grad_qmass=gq, grad_dmass=gd)
        runs.append([v.cpu().numpy() for v in (gX, gq, gd)])
    for a, b in zip(*runs):
        assert np.array_equal(a.view(np.int32), b.view(np.int32))
    want, wX, wq, wd = oracle_weighted_grad(ds, pq, pd, g_out.cpu().numpy().astype(np.float64))
    assert_grads_close(*runs[0], wX, wq, wd)
    bad = g_out.clone()
    bad[7] = float("nan")
    with pytest.raises(ft.FtError, match="finite"):
        ft.flowtree_cost_grad(ix, X, qo, qi, qm, t(pq), t(pd), ft.FT_BWD, grad_out=bad, grad_X=torch.zeros_like(X))


def test_autograd_function(ft):
    """FlowtreeCost through torch.autograd: the forward values and the
    gradients in X, q_w and d_w of sum_p g_p cost_p (g non-uniform) against
    the oracle's Flowtree and its float64 frozen gradient; a second forward
    on other pairs between a forward and its backward changes nothing; q_w
    and d_w that do not equal the masses / 2^Q are rejected."""
    say("autograd: FlowtreeCost values and gradients against the oracle")
    from paper_1910_04126_amd.autograd import flowtree_cost
    ds = gen.make("grad", V=2000, n_pairs=12)
    ix = build_index(ft, ds)
    qo, qi, qm = queries(ds)
    pq_h = np.concatenate([np.arange(12), [4]]).astype(np.int64)
    pd_h = np.concatenate([np.roll(np.arange(12), 5), [9]]).astype(np.int64)
    pq, pd = t(pq_h), t(pd_h)
    X = t(ds.X).requires_grad_(True)
    qw = (t(ds.q_mass.astype(np.float64)) * 2.0 ** -ds.Q).to(torch.float32).requires_grad_(True)
    dw = (t(ds.doc_mass.astype(np.float64)) * 2.0 ** -ds.Q).to(torch.float32).requires_grad_(True)
    g = torch.linspace(-0.7, 1.9, len(pq_h), device=X.device, dtype=torch.float32)
    c = flowtree_cost(X, qw, dw, ix, qo, qi, qm, pq, pd)
    # another forward, on a different pair list, before the first backward
    other = flowtree_cost(X, qw, dw, ix, qo, qi, qm, pq.flip(0)[:5].contiguous(), pd[:5].contiguous())
    assert other.shape == (5,)
    (c * g).sum().backward()
    want, wX, wq, wd = oracle_weighted_grad(ds, pq_h, pd_h, g.cpu().numpy().astype(np.float64))
    got = c.detach().cpu().numpy()
    assert (np.abs(got - want) <= 1e-5 * want).all()
    assert qw.grad.dtype == torch.float32 and dw.grad.dtype == torch.float32
    assert_grads_close(X.grad.cpu().numpy(), qw.grad.cpu().numpy(), dw.grad.cpu().numpy(), wX, wq, wd)
    assert np.abs(wq).max() > 0 and np.abs(wd).max() > 0
    # weights that are not the masses / 2^Q
    bad_d = dw.detach().clone()
    bad_d[3] += 2.0 ** -ds.Q
    with pytest.raises(ValueError, match="d_w"):
        flowtree_cost(X, qw, bad_d, ix, qo, qi, qm, pq, pd)
    bad_q = qw.detach().clone()
    bad_q[0] *= 0.5
    with pytest.raises(ValueError, match="q_w"):
        flowtree_cost(X, bad_q, dw, ix, qo, qi, qm, pq, pd)
    with pytest.raises(ValueError, match="d_w"):
        flowtree_cost(X, qw, dw[:-1], ix, qo, qi, qm, pq, pd)


# ------------------------------------------------------------------ errors --

def test_invalid_inputs(ft):
    say("errors: invalid inputs are rejected")
    ds = world_tiny()
    ix = build_index(ft, ds)
    qo, qi, qm = queries(ds)
    bad = qi.clone()
    bad[0] = ds.V
    with pytest.raises(ft.FtError) as e:
        ft.flowtree_knn(ix, qo, bad, qm, 5)
    assert e.value.status == -1
    bad = qm.clone()
    bad[0] += 1
    with pytest.raises(ft.FtError) as e:
        ft.quadtree_knn(ix, qo, qi, bad, 5)
    assert e.value.status == -1
    bad = qi.clone()
    bad[1] = bad[0]
    with pytest.raises(ft.FtError):
        ft.flowtree_knn(ix, qo, bad, qm, 5)
    with pytest.raises(ft.FtError):
        ft.flowtree_knn(ix, qo, qi, qm, ds.n_docs + 1)
    big = 1100
    o = torch.tensor([0, big], dtype=torch.int64, device=qo.device)
    ids = torch.arange(big, dtype=torch.int32, device=qo.device)
    m = torch.full((big,), 0, dtype=torch.int32, device=qo.device)
    m[:] = (1 << ds.Q) // big
    m[0] += (1 << ds.Q) - int(m.sum().item())
    with pytest.raises(ft.FtError) as e:
        ft.flowtree_knn(ix, o, ids, m, 5)
    assert e.value.status == -4
    # the index still works afterwards
    c, d = ft.flowtree_knn(ix, qo, qi, qm, 5)
    assert torch.isfinite(c).all()


# ------------------------------------------------------------ random model --

@pytest.mark.parametrize("N,s,eps,reps", [(100, 10, 0.25, 6), (150, 100, 0.4, 2)])
def test_random_model_against_oracle(ft, N, s, eps, reps):
    """The random-model experiment (planted doc against its single-swap
    neighbours): the top-2 of both estimates and the success flags match
    the oracle; whenever no smallest common cell H_k of (x_k, y_k) holds
    another planted point, the Flowtree value of the planted doc is the
    planted matching's cost (the event of the analysis of Section 3.2)."""
    rng = np.random.default_rng(77 + N + s)
    for rep in range(reps):
        say("random model N=%d s=%d eps=%.2f rep %d" % (N, s, eps, rep))
        ds = gen.random_model_swaps(rng, N, 10, s, eps)
        ix = build_index(ft, ds)
        T = oracle_tree(ds)
        docs = np.arange(ds.n_docs)
        keys, kd = ft.quadtree_knn(ix, *queries(ds), 2)
        costs, fd = ft.flowtree_knn(ix, *queries(ds), 2, mode=ft.FT_PLAIN)
        M = oracle_matrix(T, ds, [0], docs, "qt")[0]
        F = oracle_matrix(T, ds, [0], docs, "ft")[0]
        check_topk(kd[0].cpu().numpy(), keys[0].cpu().numpy().view(np.uint64), M, docs, 2, exact=True)
        check_topk(fd[0].cpu().numpy(), costs[0].cpu().numpy(), F, docs, 2)
        x, y = ds.extra["planted"].astype(np.int64), ds.q_id.astype(np.int64)
        event = True
        for k in range(s):
            depth = T.lca_depth(int(x[k]), int(y[k]))
            if any(T.lca_depth(int(x[j]), int(x[k])) >= depth for j in range(s) if j != k):
                event = False
        if event:
            want = float(np.mean(np.linalg.norm(ds.X[x].astype(np.float64) - ds.X[y].astype(np.float64), axis=1)))
            c = torch.empty(1, dtype=torch.float32, device="cuda")
            zero = t(np.zeros(1, np.int64))
            ft.flowtree_cost_grad(ix, t(ds.X), *queries(ds), zero, zero, ft.FT_FWD, cost=c)
            got = float(c.cpu().numpy()[0])
            assert abs(got - want) <= 1e-5 * want, "planted Flowtree %r vs matching cost %r" % (got, want)


# ------------------------------------------------------- long-row select --

@pytest.mark.parametrize("n_docs", [6000, 6001, 6003])
def test_long_rows_select(ft, n_docs):
    """Rows of 6000 keys are read four keys per load; rows of 6001 and 6003
    keys (not a multiple of four) one key per load."""
    say("select: %d docs ranked in full (window select), quadtree and flowtree" % n_docs)
    ds = gen.make("text", V=4000, d=64, n_docs=n_docs, n_queries=3)
    ix = build_index(ft, ds)
    T = oracle_tree(ds)
    docs = np.arange(ds.n_docs)
    keys, kd = ft.quadtree_knn(ix, *queries(ds), 300)
    M = oracle_matrix(T, ds, range(3), docs, "qt")
    for q in range(3):
        check_topk(kd[q].cpu().numpy(), keys[q].cpu().numpy().view(np.uint64), M[q], docs, 300, exact=True)
    c, d = ft.flowtree_knn(ix, *queries(ds), 50, mode=ft.FT_BATCHED)
    F = oracle_matrix(T, ds, range(3), docs, "ft")
    for q in range(3):
        check_topk(d[q].cpu().numpy(), c[q].cpu().numpy(), F[q], docs, 50)


@pytest.mark.parametrize("reps", [1500, 2040, 2600])
def test_long_rows_tie_bucket_sizes(ft, reps):
    """Tie buckets just below, at and above the LDS capacity of the window
    select (2048 entries)."""
    say("select: %d identical docs among %d" % (reps, reps + 4200))
    base = gen.make("tiny", n_docs=4200, n_queries=2)
    one = base.doc_id[base.doc_off[3]:base.doc_off[4]]
    onem = base.doc_mass[base.doc_off[3]:base.doc_off[4]]
    sizes = np.concatenate([np.diff(base.doc_off), np.full(reps, len(one))])
    off = np.zeros(len(sizes) + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    ids = np.concatenate([base.doc_id, np.tile(one, reps)])
    m = np.concatenate([base.doc_mass, np.tile(onem, reps)])
    ds = gen.Dataset("ties", base.X, base.shift, base.B, base.Q, off, ids, m, base.q_off, base.q_id, base.q_mass, 5)
    ix = build_index(ft, ds)
    T = oracle_tree(ds)
    docs = np.arange(ds.n_docs)
    M = oracle_matrix(T, ds, range(2), docs, "qt")
    for q in range(2):
        kth = np.sort(M[q])
        # choose k so that the k-th key is the duplicated one when possible
        dup_key = M[q][-1]
        k = int(min(1024, max(1, (M[q] < dup_key).sum() + 1)))
        keys, kd = ft.quadtree_knn(ix, *queries(ds), k)
        check_topk(kd[q].cpu().numpy(), keys[q].cpu().numpy().view(np.uint64), M[q], docs, k, exact=True)


def test_long_rows_refined_bucket(ft):
    """Thousands of distinct keys packed next to the query: the first digit
    histogram puts them all in one bucket larger than the LDS tie buffer, and
    the select must refine into the next digits instead of giving up."""
    say("select: 3000 near-duplicates of the query among 7200 docs (digit refinement)")
    base = gen.make("tiny", n_docs=4200, n_queries=2)
    one = base.doc_id[base.doc_off[3]:base.doc_off[4]]
    onem = base.doc_mass[base.doc_off[3]:base.doc_off[4]].astype(np.int64)
    reps = 3000
    var = np.tile(onem, (reps, 1))
    delta = np.arange(1, reps + 1)
    assert onem[0] > reps
    var[:, 0] -= delta  # move delta mass units from the first point to the second
    var[:, 1] += delta
    sizes = np.concatenate([np.diff(base.doc_off), np.full(reps, len(one))])
    off = np.zeros(len(sizes) + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    ids = np.concatenate([base.doc_id, np.tile(one, reps)])
    m = np.concatenate([base.doc_mass, var.reshape(-1).astype(np.uint32)])
    q_off = np.array([0, len(one), len(one) + base.q_off[1]], np.int64)
    q_id = np.concatenate([one, base.q_id[:base.q_off[1]]])
    q_m = np.concatenate([onem.astype(np.uint32), base.q_mass[:base.q_off[1]]])
    ds = gen.Dataset("near", base.X, base.shift, base.B, base.Q, off, ids, m, q_off, q_id, q_m, 5)
    ix = build_index(ft, ds)
    T = oracle_tree(ds)
    docs = np.arange(ds.n_docs)
    M = oracle_matrix(T, ds, range(2), docs, "qt")
    for k in (1000, 1024):
        keys, kd = ft.quadtree_knn(ix, *queries(ds), k)
        for q in range(2):
            check_topk(kd[q].cpu().numpy(), keys[q].cpu().numpy().view(np.uint64), M[q], docs, k, exact=True)


def test_long_rows_many_ties(ft):
    """Thousands of identical docs give thousands of equal keys at the k-th
    position: the one-pass gather overflows, the exact path's bucket of the
    k-th key stays too large to refine, and the in-order scan over the equal
    keys must give the ties to the lowest doc indices."""
    say("select: 5000 docs, 4200 identical (in-order tie scan)")
    base = gen.make("tiny", n_docs=800, n_queries=2)
    reps = 4200
    one = base.doc_id[base.doc_off[0]:base.doc_off[1]]
    onem = base.doc_mass[base.doc_off[0]:base.doc_off[1]]
    sizes = np.concatenate([np.full(reps, len(one)), np.diff(base.doc_off)])
    off = np.zeros(len(sizes) + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    ids = np.concatenate([np.tile(one, reps), base.doc_id])
    m = np.concatenate([np.tile(onem, reps), base.doc_mass])
    ds = gen.Dataset("ties", base.X, base.shift, base.B, base.Q, off, ids, m, base.q_off, base.q_id, base.q_mass, 5)
    ix = build_index(ft, ds)
    T = oracle_tree(ds)
    docs = np.arange(ds.n_docs)
    M = oracle_matrix(T, ds, range(2), docs, "qt")
    F = oracle_matrix(T, ds, range(2), docs, "ft")
    for k in (1000, 1024):
        keys, kd = ft.quadtree_knn(ix, *queries(ds), k)
        for q in range(2):
            check_topk(kd[q].cpu().numpy(), keys[q].cpu().numpy().view(np.uint64), M[q], docs, k, exact=True)
    c, d = ft.flowtree_knn(ix, *queries(ds), 1000, mode=ft.FT_BATCHED)
    for q in range(2):
        check_topk(d[q].cpu().numpy(), c[q].cpu().numpy(), F[q], docs, 1000)
