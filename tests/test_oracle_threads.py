"""The oracle as the all-cores CPU baseline runs it: one tree per thread,
calls from several threads at once (the C calls release the GIL).  Values
must equal those of one thread, bit for bit."""
import threading

import numpy as np

import gen
import oracle


def test_threads_with_own_trees_match_one_thread():
    ds = gen.make("tiny", seed=9, n_docs=400, n_queries=8)
    docs = np.arange(ds.n_docs)

    def run(Tr, q):
        pq = np.full(ds.n_docs, q)
        U = Tr.quadtree_pairs(ds.q_off, ds.q_id, ds.q_mass, ds.doc_off, ds.doc_id, ds.doc_mass, pq, docs, ds.Q)
        F = Tr.flowtree_pairs(ds.q_off, ds.q_id, ds.q_mass, ds.doc_off, ds.doc_id, ds.doc_mass, pq, docs, ds.Q)
        return U, F

    one = oracle.Tree(ds.X, ds.shift, ds.B)
    want = [run(one, q) for q in range(ds.n_queries)]
    got = [None] * ds.n_queries
    trees = [oracle.Tree(ds.X, ds.shift, ds.B) for _ in range(4)]

    def worker(i):
        for rep in range(3):
            for q in range(i, ds.n_queries, 4):
                got[q] = run(trees[i], q)

    ths = [threading.Thread(target=worker, args=(i,)) for i in range(4)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    for q in range(ds.n_queries):
        assert np.array_equal(got[q][0], want[q][0])
        assert np.array_equal(got[q][1].view(np.int64), want[q][1].view(np.int64))
