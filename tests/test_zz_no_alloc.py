"""ft_flowtree_knn_noalloc, the entry point that allocates nothing: its output
must equal ft_flowtree_knn's (same candidates) bit for bit, on two calls in a
row, the second with a smaller input, and its size limits must be refused
before any device work."""
import numpy as np
import pytest
import torch

import gen
from gpu_util import build_index, queries, t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ft():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1910_04126_amd as ft
    ft.load()
    return ft


def _cands(rng, n_q, n_docs, n_cand):
    return np.stack([rng.choice(n_docs, n_cand, replace=False) for _ in range(n_q)]).astype(np.int64)


def _case(ft, ix, ds, sel, cand, k):
    qo, qi, qm = queries(ds, sel)
    ct = t(cand)
    print("noalloc case: %d queries x %d candidates, k=%d" % (len(sel), cand.shape[1], k), flush=True)
    na_c, na_d = ft.flowtree_knn_noalloc(ix, qo, qi, qm, k, ct)
    ref_c, ref_d = ft.flowtree_knn(ix, qo, qi, qm, k, cand=ct, mode=ft.FT_BATCHED)
    torch.cuda.synchronize()
    assert torch.equal(na_d, ref_d)
    assert torch.equal(na_c.view(torch.int32), ref_c.view(torch.int32))
    return na_c, na_d


@pytest.mark.parametrize("name", ["tiny", "batched"])
def test_noalloc_matches_flowtree_knn_twice(ft, name):
    if name == "tiny":
        ds = gen.make("tiny", seed=3, n_docs=500, n_queries=12)
        big, small = (12, 400, 9), (5, 37, 3)
    else:
        # text-shaped sizes 5..500: pairs reach the 1024-item class
        ds = gen.make("batched", seed=4, V=20_000, n_docs=3000, n_queries=48)
        big, small = (48, 700, 20), (7, 129, 5)
    ix = build_index(ft, ds)
    rng = np.random.default_rng(11)
    nq, nc, k = big
    _case(ft, ix, ds, np.arange(nq), _cands(rng, nq, ds.n_docs, nc), k)
    nq, nc, k = small
    sel = rng.choice(ds.n_queries, nq, replace=False)
    _case(ft, ix, ds, sel, _cands(rng, nq, ds.n_docs, nc), k)


def test_noalloc_limits_and_errors(ft):
    ds = gen.make("tiny", seed=5, n_docs=300, n_queries=4)
    ix = build_index(ft, ds)
    qo, qi, qm = queries(ds)
    rng = np.random.default_rng(2)
    cand = t(_cands(rng, 4, ds.n_docs, 50))
    # k out of range and n_cand beyond 4096: refused on the host
    with pytest.raises(ft.FtError) as e:
        ft.flowtree_knn_noalloc(ix, qo, qi, qm, 51, cand)
    assert e.value.status == -1
    # more pairs than the scratch array holds: refused on the host
    many = gen.make("tiny", seed=6, n_docs=300, n_queries=300)
    mo, mi, mm = queries(many)
    big = torch.zeros((300, 4000), dtype=torch.int64, device=mo.device)
    with pytest.raises(ft.FtError) as e:
        ft.flowtree_knn_noalloc(ix, mo, mi, mm, 5, big)
    assert e.value.status == -4 and "FT_NOALLOC_MAX_PAIRS" in str(e.value)
    # more query items than the scratch array holds (the offsets are read
    # first, nothing else is touched)
    long = gen.make("tiny", seed=7, n_docs=300, n_queries=1100, lo=250, hi=260)
    lo_, li, lm = queries(long)
    with pytest.raises(ft.FtError) as e:
        ft.flowtree_knn_noalloc(ix, lo_, li, lm, 1, torch.zeros((1100, 1), dtype=torch.int64, device=lo_.device))
    assert e.value.status == -4 and "FT_NOALLOC_MAX_ITEMS" in str(e.value)
    # a candidate out of range: FT_EINVAL from the device check
    badc = cand.clone()
    badc[1, 3] = ds.n_docs
    with pytest.raises(ft.FtError) as e:
        ft.flowtree_knn_noalloc(ix, qo, qi, qm, 5, badc)
    assert e.value.status == -1
    # the shared status words were left set by that call; the next one clears them
    _case(ft, ix, ds, np.arange(4), cand.cpu().numpy(), 5)
