"""The oracle's CSR batch helpers against the single-pair functions they wrap.

Every GPU cost comparison goes through ``Tree.quadtree_pairs``,
``Tree.flowtree_pairs``, ``oracle.act_pairs`` and ``oracle.sinkhorn_pairs``.
Each one only slices a query and a dataset distribution out of two CSR sets
and calls the single-pair estimate with the dataset side as mu and the query
side as nu (the orientation of Section 3's Flowtree definition, where the
query is compared against each dataset distribution).  The single-pair
functions are pinned elsewhere against the paper (closed forms, LPs, hand
values); this file pins the slicing: uneven CSR sets of different lengths,
pair lists in shuffled order with repeats, pair_q != pair_d, and the empty
pair list.  An off-by-one in an offset, a query index used on the dataset
side, or a swapped orientation (Sinkhorn is not symmetric) fails here.
"""
import numpy as np
import pytest

import gen
import oracle

Q = 20


def _csr(rng, n, V, lo, hi):
    """n distributions with supports of lo..hi distinct ids and random
    positive integer masses summing to 2^Q."""
    sizes = rng.integers(lo, hi + 1, size=n)
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    ids, ms = [], []
    for s in sizes:
        ids.append(np.sort(rng.choice(V, size=s, replace=False)).astype(np.uint32))
        cuts = np.sort(rng.choice(np.arange(1, 1 << Q), size=s - 1, replace=False))
        ms.append(np.diff(np.concatenate([[0], cuts, [1 << Q]])).astype(np.uint32))
    return off, np.concatenate(ids), np.concatenate(ms)


@pytest.fixture(scope="module")
def world():
    rng = np.random.default_rng(11)
    V, d = 300, 5
    X = gen.gaussian_mixture(rng, V, d, 6, 0.3, normalize=False)
    shift = gen.random_shift(rng, d)
    T = oracle.Tree(X, shift)
    q = _csr(rng, 7, V, 1, 13)       # 7 queries
    ds = _csr(rng, 11, V, 1, 17)     # 11 dataset distributions
    n = 60
    pair_q = rng.integers(0, 7, size=n).astype(np.int64)
    pair_d = rng.integers(0, 11, size=n).astype(np.int64)
    pair_q[:3] = [6, 0, 6]           # repeats and both ends of each set
    pair_d[:3] = [10, 0, 10]
    return X, T, q, ds, pair_q, pair_d


def _slices(q, ds, i, j):
    (qo, qi, qm), (do, di, dm) = q, ds
    return (di[do[j]:do[j + 1]], dm[do[j]:do[j + 1]], qi[qo[i]:qo[i + 1]], qm[qo[i]:qo[i + 1]])


def test_sets_are_uneven(world):
    _, _, q, ds, pq, pd = world
    assert len(set(np.diff(q[0]).tolist())) > 3 and len(set(np.diff(ds[0]).tolist())) > 3
    assert (pq != pd).sum() > 40


def test_quadtree_pairs_match_single(world):
    _, T, q, ds, pq, pd = world
    got = T.quadtree_pairs(*q, *ds, pq, pd, Q)
    want = [T.quadtree(*_slices(q, ds, i, j), Q=Q) for i, j in zip(pq, pd)]
    assert [int(v) for v in got] == want


def test_flowtree_pairs_match_single(world):
    _, T, q, ds, pq, pd = world
    got = T.flowtree_pairs(*q, *ds, pq, pd, Q)
    want = [T.flowtree(*_slices(q, ds, i, j), Q=Q)[0] for i, j in zip(pq, pd)]
    assert got.tolist() == want          # same arithmetic, bit-identical


@pytest.mark.parametrize("iters", [0, 1, 3])
def test_act_pairs_match_single(world, iters):
    X, _, q, ds, pq, pd = world
    got = oracle.act_pairs(X, *q, *ds, pq, pd, Q, iters)
    want = [oracle.act(X, *_slices(q, ds, i, j), Q, iters) for i, j in zip(pq, pd)]
    assert got.tolist() == want


@pytest.mark.parametrize("iters", [1, 3])
def test_sinkhorn_pairs_match_single(world, iters):
    X, _, q, ds, pq, pd = world
    got = oracle.sinkhorn_pairs(X, *q, *ds, pq, pd, Q, iters, 30.0)
    want = [oracle.sinkhorn(X, *_slices(q, ds, i, j), Q, iters, 30.0) for i, j in zip(pq, pd)]
    assert got.tolist() == want


def test_sinkhorn_orientation_matters(world):
    """The helper's orientation is observable: Sinkhorn-1 with mu and nu
    swapped differs on some pair, so the test above would catch a swap."""
    X, _, q, ds, pq, pd = world
    diff = 0
    for i, j in zip(pq[:20], pd[:20]):
        mu_id, mu_m, nu_id, nu_m = _slices(q, ds, i, j)
        a = oracle.sinkhorn(X, mu_id, mu_m, nu_id, nu_m, Q, 1, 30.0)
        b = oracle.sinkhorn(X, nu_id, nu_m, mu_id, mu_m, Q, 1, 30.0)
        diff += abs(a - b) > 1e-9 * max(a, b)
    assert diff > 0


def test_empty_pair_list(world):
    X, T, q, ds, _, _ = world
    e = np.zeros(0, np.int64)
    assert T.quadtree_pairs(*q, *ds, e, e, Q).shape == (0,)
    assert T.flowtree_pairs(*q, *ds, e, e, Q).shape == (0,)
    assert oracle.act_pairs(X, *q, *ds, e, e, Q, 1).shape == (0,)
    assert oracle.sinkhorn_pairs(X, *q, *ds, e, e, Q, 1).shape == (0,)


# Plausible slips in the C batch helpers, each planted in a copy of oracle.c:
# the comparisons above must catch every one.
BATCH_MUTANTS = {
    "quadtree: doc slice taken with the query index": (
        "int64_t da = d_off[pair_d[p]], db = d_off[pair_d[p] + 1];\n"
        "    int rc = oracle_quadtree(",
        "int64_t da = d_off[pair_q[p]], db = d_off[pair_q[p] + 1];\n"
        "    int rc = oracle_quadtree("),
    "quadtree: query slice one item short": (
        "int rc = oracle_quadtree(t, d_id + da, d_m + da, db - da, q_id + qa, q_m + qa,\n"
        "                             qb - qa, Q, out + p);",
        "int rc = oracle_quadtree(t, d_id + da, d_m + da, db - da, q_id + qa, q_m + qa,\n"
        "                             qb - qa - (qb - qa > 1), Q, out + p);"),
    "flowtree: doc slice starts one item late": (
        "rc = oracle_flowtree(t, X, d_id + da, d_m + da, db - da,",
        "rc = oracle_flowtree(t, X, d_id + da + (db - da > 1), d_m + da + (db - da > 1),"
        " db - da - (db - da > 1),"),
}


def _batch_checks_pass(lib, world):
    X, _, q, ds, pq, pd = world
    T = oracle.Tree(X, world[1].shift, lib=lib)
    try:
        got_u = T.quadtree_pairs(*q, *ds, pq, pd, Q)
        got_f = T.flowtree_pairs(*q, *ds, pq, pd, Q)
    except oracle.OracleError:
        return False
    want_u = [T.quadtree(*_slices(q, ds, i, j), Q=Q) for i, j in zip(pq, pd)]
    want_f = [T.flowtree(*_slices(q, ds, i, j), Q=Q)[0] for i, j in zip(pq, pd)]
    return [int(v) for v in got_u] == want_u and got_f.tolist() == want_f


def test_batch_checks_pass_on_oracle(world):
    assert _batch_checks_pass(oracle._lib(), world)


@pytest.mark.parametrize("name", sorted(BATCH_MUTANTS))
def test_batch_checks_catch_mutant(name, world, tmp_path):
    from test_oracle_mutants import build_variant
    old, new = BATCH_MUTANTS[name]
    lib = build_variant(str(tmp_path), old, new)
    assert not _batch_checks_pass(lib, world), "batch checks did not catch: " + name
