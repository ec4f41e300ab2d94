"""ft_knn_pipeline: the Quadtree prune of every doc followed by the batched
Flowtree rerank in one call (the two-stage search of Section 4.3).  Its
output must equal the two calls it replaces bit for bit, on datasets that
take either ranking path of the prune (all docs fit one select block, or not),
and its argument limits must be refused before any device work."""
import numpy as np
import pytest
import torch

import gen
from gpu_util import build_index, check_topk, oracle_matrix, oracle_tree, queries, t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ft():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1910_04126_amd as ft
    ft.load()
    return ft


@pytest.mark.parametrize("name,prune,k", [("tiny", 60, 7), ("batched", 300, 20)])
def test_pipeline_equals_two_calls(ft, name, prune, k):
    if name == "tiny":
        ds = gen.make("tiny", seed=21, n_docs=800, n_queries=10)
    else:
        ds = gen.make("batched", seed=22, V=20_000, n_docs=9000, n_queries=40)
    print("pipeline case %s: %d docs, %d queries, prune %d, k %d" % (name, ds.n_docs, ds.n_queries, prune, k),
          flush=True)
    ix = build_index(ft, ds)
    qo, qi, qm = queries(ds)
    for rep in range(2):
        keys, cand = ft.quadtree_knn(ix, qo, qi, qm, prune)
        c2, d2 = ft.flowtree_knn(ix, qo, qi, qm, k, cand=cand, mode=ft.FT_BATCHED)
        c1, d1 = ft.knn_pipeline(ix, qo, qi, qm, prune, k)
        torch.cuda.synchronize()
        assert torch.equal(d1, d2)
        assert torch.equal(c1.view(torch.int32), c2.view(torch.int32))
    pr, rr = ix.last_pipeline_stats()
    assert pr > 0.0 and rr > 0.0
    # one sampled query against the oracle: the pipeline's answer is the
    # Flowtree top-k of the oracle's exact Quadtree top-prune
    T = oracle_tree(ds)
    q = ds.n_queries - 1
    all_docs = np.arange(ds.n_docs)
    M = oracle_matrix(T, ds, [q], all_docs, "qt")[0]
    order = np.lexsort((all_docs, M))[:prune]
    assert np.array_equal(np.sort(order), np.sort(cand[q].cpu().numpy()))
    F = oracle_matrix(T, ds, [q], order, "ft")[0]
    swaps = check_topk(d1[q].cpu().numpy(), c1[q].cpu().numpy(), F, order, k)
    assert swaps <= 1


def test_pipeline_limits(ft):
    ds = gen.make("tiny", seed=23, n_docs=5000, n_queries=3)
    ix = build_index(ft, ds)
    qo, qi, qm = queries(ds)
    for prune, k, what in ((0, 1, "prune_k must lie"), (5001, 1, "prune_k must lie"),
                           (2000, 5, "prune_k > 1024 needs at most 4096 docs"), (10, 11, "k must lie")):
        with pytest.raises(Exception, match=what):
            ft.knn_pipeline(ix, qo, qi, qm, prune, k)
    c, d = ft.knn_pipeline(ix, qo, qi, qm, 1024, 3)
    torch.cuda.synchronize()
    assert d.shape == (3, 3)
