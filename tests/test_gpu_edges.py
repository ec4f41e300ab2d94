"""Degenerate ground sets through the whole path.

* Phi = 0: every point coincides (Section 2: the enclosing cube has side 0,
  so no halving ever separates two points).  The tree is one chain of cells
  down to a single depth-B leaf holding all V points, every Quadtree value is
  0 (each cell on the chain holds all the mass of both distributions) and
  every Flowtree value is 0 (each match joins two copies of one location).
* V = 1: the root itself is the only leaf (it holds exactly one point), the
  tree has height 0, and every distribution is the point mass on it.

The CPU tests pin the oracle on both (the values are fixed by the
definitions, not by the oracle).  The GPU tests run the library on them and
compare bit for bit: tree arrays, Quadtree keys over all docs and over
candidate lists, plain and batched Flowtree, the flow triples, and the
forward / backward of the frozen cost.
"""
import sys

import numpy as np
import pytest

import gen
import oracle
from gpu_util import build_index, oracle_flow_set, queries, t

Q = 24
B = 30


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _uniform_sets(V, sizes, seed):
    rng = np.random.default_rng(seed)
    off = np.zeros(len(sizes) + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    ids = np.concatenate([np.sort(rng.choice(V, s, replace=False)) for s in sizes]).astype(np.uint32)
    return off, ids, gen.uniform_masses(off, ids, Q)


def world_phi0(V, d, seed):
    """V coincident points in R^d; 9 docs and 4 queries of 1..V points."""
    X = np.full((V, d), 0.25, np.float32)
    rng = np.random.default_rng(seed)
    shift = gen.random_shift(rng, d, B)
    do, di, dm = _uniform_sets(V, rng.integers(1, V + 1, size=9), seed + 1)
    qo, qi, qm = _uniform_sets(V, rng.integers(1, V + 1, size=4), seed + 2)
    return gen.Dataset("phi0", X, shift, B, Q, do, di, dm, qo, qi, qm, 3)


def world_v1():
    """One ground point; 5 docs and 3 queries, all the point mass on it."""
    X = np.array([[0.5, -1.0, 2.0]], np.float32)
    one = lambda n: (np.arange(n + 1, dtype=np.int64), np.zeros(n, np.uint32),
                     np.full(n, 1 << Q, np.uint32))
    do, di, dm = one(5)
    qo, qi, qm = one(3)
    return gen.Dataset("v1", X, np.array([7, 1, 3]), B, Q, do, di, dm, qo, qi, qm, 3)


WORLDS = {"phi0_2d": lambda: world_phi0(4, 2, 3), "phi0_32d": lambda: world_phi0(6, 32, 4),
          "v1": world_v1}


def all_pairs(ds):
    pq = np.repeat(np.arange(ds.n_queries), ds.n_docs).astype(np.int64)
    pd = np.tile(np.arange(ds.n_docs), ds.n_queries).astype(np.int64)
    return pq, pd


# ------------------------------------------------------ oracle (CPU) pins --

@pytest.mark.parametrize("name", sorted(WORLDS))
def test_oracle_tree_shape(name):
    ds = WORLDS[name]()
    T = oracle.Tree(ds.X, ds.shift, ds.B)
    ex = T.export()
    assert T.phi == 0.0
    if ds.V == 1:
        assert T.n_nodes == 1 and ex["leaf_depth"].tolist() == [0]
    else:
        # the root and one cell per depth down to the depth-B leaf
        assert T.n_nodes == B + 1
        assert ex["leaf_depth"].tolist() == [B] * ds.V
        assert ex["rank_of"].tolist() == list(range(ds.V))  # by id inside the leaf


@pytest.mark.parametrize("name", sorted(WORLDS))
def test_oracle_values_are_zero(name):
    ds = WORLDS[name]()
    T = oracle.Tree(ds.X, ds.shift, ds.B)
    pq, pd = all_pairs(ds)
    U = T.quadtree_pairs(ds.q_off, ds.q_id, ds.q_mass, ds.doc_off, ds.doc_id, ds.doc_mass, pq, pd, Q)
    F = T.flowtree_pairs(ds.q_off, ds.q_id, ds.q_mass, ds.doc_off, ds.doc_id, ds.doc_mass, pq, pd, Q)
    assert (U == 0).all() and (F == 0.0).all()


# --------------------------------------------------------- GPU parity ------

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ft():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_04126_amd as m
    m.load()
    return m


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(WORLDS))
def test_gpu_tree(ft, name):
    say("edges: tree of", name)
    ds = WORLDS[name]()
    ix = build_index(ft, ds)
    T = oracle.Tree(ds.X, ds.shift, ds.B)
    ex = T.export()
    perm, lcp, ld = [v.cpu().numpy().astype(np.int64) for v in ix.export_tree()]
    assert perm.tolist() == np.argsort(ex["rank_of"]).tolist()
    assert ld.tolist() == ex["leaf_depth"][perm].tolist()
    assert lcp.tolist() == [B] * (ds.V - 1) + [0]
    info = ix.info()
    assert info["height"] == ex["leaf_depth"].max() and info["n_nodes"] == T.n_nodes


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(WORLDS))
def test_gpu_quadtree_zero(ft, name):
    say("edges: quadtree keys of", name)
    ds = WORLDS[name]()
    ix = build_index(ft, ds)
    qo, qi, qm = queries(ds)
    k = ds.n_docs
    keys, docs = ft.quadtree_knn(ix, qo, qi, qm, k)
    assert (keys.cpu() == 0).all()
    assert docs.cpu().tolist() == [list(range(k))] * ds.n_queries  # ties by doc index
    cand = torch.tensor([list(range(ds.n_docs))[::-1]] * ds.n_queries, dtype=torch.int64, device=qo.device)
    keys, docs = ft.quadtree_knn(ix, qo, qi, qm, 2, cand=cand)
    assert (keys.cpu() == 0).all() and docs.cpu().tolist() == [[0, 1]] * ds.n_queries
    pq, pd = all_pairs(ds)
    assert (ft.quadtree_pairs(ix, qo, qi, qm, t(pq), t(pd)).cpu() == 0).all()


@pytest.mark.gpu
@pytest.mark.parametrize("mode", ["plain", "batched"])
@pytest.mark.parametrize("name", sorted(WORLDS))
def test_gpu_flowtree_zero(ft, name, mode):
    say("edges: flowtree", mode, "of", name)
    ds = WORLDS[name]()
    ix = build_index(ft, ds)
    qo, qi, qm = queries(ds)
    m = ft.FT_PLAIN if mode == "plain" else ft.FT_BATCHED
    cost, docs = ft.flowtree_knn(ix, qo, qi, qm, ds.n_docs, mode=m)
    assert (cost.cpu() == 0).all()
    assert docs.cpu().tolist() == [list(range(ds.n_docs))] * ds.n_queries
    cand = torch.tensor([[4, 2, 0]] * ds.n_queries, dtype=torch.int64, device=qo.device)
    cost, docs = ft.flowtree_knn(ix, qo, qi, qm, 3, cand=cand, mode=m)
    assert (cost.cpu() == 0).all() and docs.cpu().tolist() == [[0, 2, 4]] * ds.n_queries


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(WORLDS))
def test_gpu_flows_bitexact(ft, name):
    say("edges: flows of", name)
    ds = WORLDS[name]()
    ix = build_index(ft, ds)
    T = oracle.Tree(ds.X, ds.shift, ds.B)
    pq, pd = all_pairs(ds)
    flows = ft.flowtree_flows(ix, *queries(ds), t(pq), t(pd))
    for (q, doc), (fd, fq, fe, fb) in zip(zip(pq, pd), flows):
        got = sorted(zip(fd.tolist(), fq.tolist(), fe.tolist(), fb.tolist()))
        assert got == oracle_flow_set(T, ds, q, doc)
    if ds.V == 1:
        assert all(len(f[0]) == 1 and int(f[2][0]) == 1 << Q and int(f[3][0]) == 2 for f in flows)


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(WORLDS))
def test_gpu_cost_grad_zero(ft, name):
    """Every match joins two copies of one location: the cost is 0, D_e = 0
    gives the zero subgradient in X, and the weight adjoints (sums of D_e)
    are 0."""
    say("edges: cost and gradient of", name)
    ds = WORLDS[name]()
    ix = build_index(ft, ds)
    X = t(ds.X)
    qo, qi, qm = queries(ds)
    pq, pd = all_pairs(ds)
    cost = torch.full((len(pq),), 7.0, dtype=torch.float32, device=X.device)
    ft.flowtree_cost_grad(ix, X, qo, qi, qm, t(pq), t(pd), ft.FT_FWD, cost=cost)
    gX = torch.zeros_like(X)
    gq = torch.zeros(len(ds.q_id), device=X.device)
    gd = torch.zeros(len(ds.doc_id), device=X.device)
    g_out = torch.linspace(0.5, 2.0, len(pq), device=X.device)
    ft.flowtree_cost_grad(ix, X, qo, qi, qm, t(pq), t(pd), ft.FT_BWD, grad_out=g_out, grad_X=gX,
                          grad_qmass=gq, grad_dmass=gd)
    assert (cost.cpu() == 0).all()
    assert (gX.cpu() == 0).all() and (gq.cpu() == 0).all() and (gd.cpu() == 0).all()
