"""Helpers shared by the GPU parity tests: moving gen datasets to the device,
running the oracle on the same inputs, and the top-k comparison rule."""
import numpy as np
import torch

import oracle

RTOL_COST = 1e-5      # float32 Flowtree cost vs the float64 oracle
RTOL_TIE = 2e-5       # two docs whose oracle costs are this close may swap ranks


def dev():
    return torch.device("cuda", torch.cuda.current_device())


def t(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).to(dev())


def build_index(ft, ds):
    return ft.build_tree(t(ds.X), ds.shift, ds.B, t(ds.doc_off), t(ds.doc_id), t(ds.doc_mass), ds.Q)


def queries(ds, sel=None):
    if sel is None:
        return t(ds.q_off), t(ds.q_id), t(ds.q_mass)
    off, ids, m = subset(ds.q_off, ds.q_id, ds.q_mass, sel)
    return t(off), t(ids), t(m)


def subset(off, ids, mass, sel):
    sel = np.asarray(sel)
    sizes = off[sel + 1] - off[sel]
    o = np.zeros(len(sel) + 1, np.int64)
    o[1:] = np.cumsum(sizes)
    idx = np.concatenate([np.arange(off[j], off[j + 1]) for j in sel])
    return o, ids[idx], mass[idx]


def oracle_tree(ds):
    return oracle.Tree(ds.X, ds.shift, ds.B)


def oracle_matrix(T, ds, q_sel, docs, kind, q_csr=None):
    """Oracle values for every (query in q_sel, doc in docs): uint64 Quadtree
    keys or float64 Flowtree costs, shape [len(q_sel), len(docs)]."""
    qo, qi, qm = q_csr if q_csr is not None else (ds.q_off, ds.q_id, ds.q_mass)
    docs = np.asarray(docs, np.int64)
    out = []
    for q in q_sel:
        pq = np.full(len(docs), q, np.int64)
        f = T.quadtree_pairs if kind == "qt" else T.flowtree_pairs
        out.append(f(qo, qi, qm, ds.doc_off, ds.doc_id, ds.doc_mass, pq, docs, ds.Q))
    return np.stack(out)


def check_topk(gpu_docs, gpu_costs, oracle_costs, doc_ids, k, exact=False):
    """gpu_docs / gpu_costs: the library's ordered top-k for one query.
    oracle_costs[j] is the oracle value of candidate doc_ids[j].  Integer keys
    must give the identical ordered list.  Float costs must each lie within
    RTOL_COST of the oracle, and the ordered list must equal the oracle's
    (cost, doc) order except where the two docs at a position have oracle
    costs within RTOL_TIE (near-ties, counted and returned)."""
    doc_ids = np.asarray(doc_ids)
    order = np.lexsort((doc_ids, oracle_costs))[:k]
    want = doc_ids[order]
    lookup = {int(dd): float(c) for dd, c in zip(doc_ids, oracle_costs)}
    gpu_docs = np.asarray(gpu_docs)
    assert len(set(gpu_docs.tolist())) == k, "duplicate docs in the top-k"
    if exact:
        assert gpu_docs.tolist() == want.tolist()
        assert [int(x) for x in np.asarray(gpu_costs)] == [int(x) for x in oracle_costs[order]]
        return 0
    swaps = 0
    for i, (a, b) in enumerate(zip(gpu_docs.tolist(), want.tolist())):
        ca = lookup[a]
        assert abs(float(gpu_costs[i]) - ca) <= RTOL_COST * abs(ca) + 1e-30, \
            "cost of doc %d: gpu %r oracle %r" % (a, float(gpu_costs[i]), ca)
        if a != b:
            cb = lookup[b]
            assert abs(ca - cb) <= RTOL_TIE * max(abs(ca), abs(cb)), \
                "rank %d: gpu doc %d (%r) vs oracle doc %d (%r)" % (i, a, ca, b, cb)
            swaps += 1
    return swaps


def oracle_flow_set(T, ds, q, doc, q_csr=None):
    qo, qi, qm = q_csr if q_csr is not None else (ds.q_off, ds.q_id, ds.q_mass)
    mu_id = ds.doc_id[ds.doc_off[doc]:ds.doc_off[doc + 1]]
    mu_m = ds.doc_mass[ds.doc_off[doc]:ds.doc_off[doc + 1]]
    nu_id = qi[qo[q]:qo[q + 1]]
    nu_m = qm[qo[q]:qo[q + 1]]
    _, fl = T.flowtree(mu_id, mu_m, nu_id, nu_m, Q=ds.Q, with_cost=False)
    return sorted((int(mu_id[a]), int(nu_id[b]), int(e), int(bd))
                  for a, b, e, bd in zip(fl["mu"], fl["nu"], fl["eta"], fl["bind"]))
