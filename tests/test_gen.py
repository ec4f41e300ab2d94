"""Input generators: the laws stated in gen's docstrings hold."""
import numpy as np
import pytest

import gen


@pytest.mark.parametrize("name,over", [
    ("tiny", {}),
    ("text", dict(V=3000, n_docs=300, n_queries=20)),
    ("batched", dict(V=3000, n_docs=400, n_queries=20)),
    ("image", dict(n_docs=60, n_queries=5)),
    ("grad", dict(V=3000, n_pairs=16)),
])
def test_distributions_are_valid(name, over):
    ds = gen.make(name, seed=3, **over)
    for off, ids, m in ((ds.doc_off, ds.doc_id, ds.doc_mass), (ds.q_off, ds.q_id, ds.q_mass)):
        assert off[0] == 0 and (np.diff(off) > 0).all() and off[-1] == len(ids) == len(m)
        assert ids.max() < ds.V and m.min() >= 1
        sums = np.add.reduceat(m.astype(np.int64), off[:-1])
        assert (sums == (1 << ds.Q)).all()
        for j in range(0, len(off) - 1, max(1, (len(off) - 1) // 25)):
            sup = ids[off[j]:off[j + 1]]
            assert len(np.unique(sup)) == len(sup)
    assert ds.shift.min() >= 1 and ds.shift.max() <= (1 << (ds.B - 1))
    assert ds.X.dtype == np.float32 and np.isfinite(ds.X).all()


def test_deterministic():
    a = gen.make("tiny", seed=5)
    b = gen.make("tiny", seed=5)
    assert (a.X == b.X).all() and (a.doc_id == b.doc_id).all() and (a.shift == b.shift).all()


def test_uniform_mass_rule():
    off = np.array([0, 3, 10])
    ids = np.array([9, 2, 5, 7, 1, 8, 3, 4, 6, 0], np.uint32)
    m = gen.uniform_masses(off, ids, 4)           # 16/3 -> 5 r1 ; 16/7 -> 2 r2
    assert m[:3].tolist() == [5, 6, 5]            # id 2 is the smallest
    assert m[3:].tolist() == [2, 3, 2, 2, 2, 2, 3]  # ids 0 and 1 get +1


def test_sizes_laws():
    rng = np.random.default_rng(0)
    s = gen.sizes_power(rng, 200000, 5, 500)
    assert s.min() >= 5 and s.max() <= 500
    # P(5)/P(10) = 2**1.1
    r = (s == 5).sum() / (s == 10).sum()
    assert r == pytest.approx(2 ** 1.1, rel=0.05)


def test_random_model_cap():
    rng = np.random.default_rng(1)
    X, doc, qry = gen.random_model(rng, 50, 10, 4, 0.25)
    assert np.allclose(np.linalg.norm(X.astype(float), axis=1), 1, atol=1e-6)
    assert (np.linalg.norm(X[doc].astype(float) - X[qry], axis=1) <= 0.25 + 1e-6).all()
