"""Python binding of libftree (include/ftree.h): Quadtree and Flowtree k-NN
for Wasserstein-1 on MI355X (arXiv 1910.04126).

Argument marshalling only: every step runs in the HIP library.  Arrays are
torch CUDA tensors (contiguous); uint32 data travels in int32 tensors and
uint64 keys in int64 tensors (same bits).  The functions carry the names of
the C entry points.  Loading fails loudly when libftree.so is missing.
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = ["Index", "build_tree", "quadtree_knn", "flowtree_knn", "flowtree_knn_noalloc", "flowtree_cost_grad",
           "flowtree_flows", "quadtree_pairs", "FtError", "FT_PLAIN", "FT_BATCHED",
           "FT_FWD", "FT_BWD", "lib_path", "load"]

FT_PLAIN, FT_BATCHED = 0, 1
FT_FWD, FT_BWD = 0, 1
_STATUS = {0: "FT_OK", -1: "FT_EINVAL", -2: "FT_ENOMEM", -3: "FT_EHIP", -4: "FT_ERANGE"}

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib_path() -> str:
    return os.path.join(_HERE, "libftree.so")


class FtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


def load():
    """Load libftree.so (built by paper_1910_04126_amd.build)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError("libftree.so is not built; run python -m paper_1910_04126_amd.build")
    lib = ctypes.CDLL(path)
    p, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    sig = {
        "ft_last_error": ([], ctypes.c_char_p),
        "ft_build_tree": ([p, i64, i32, p, i32, p, p, p, i64, i32, p, ctypes.POINTER(p)], ctypes.c_int),
        "ft_free": ([p], None),
        "ft_index_info": ([p, p], ctypes.c_int),
        "ft_export_tree": ([p, p, p, p, p], ctypes.c_int),
        "ft_quadtree_knn": ([p, p, p, p, i64, p, i32, i32, p, p, p], ctypes.c_int),
        "ft_flowtree_knn": ([p, p, p, p, i64, p, i32, i32, i32, p, p, p], ctypes.c_int),
        "ft_flowtree_knn_noalloc": ([p, p, p, p, i64, p, i32, i32, p, p, p], ctypes.c_int),
        "ft_knn_pipeline": ([p, p, p, p, i64, i32, i32, p, p, p], ctypes.c_int),
        "ft_last_pipeline_stats": ([p, p, p], ctypes.c_int),
        "ft_flowtree_cost_grad": ([p, p, p, p, p, i64, p, p, i64, i32, p, p, p, p, p, p], ctypes.c_int),
        "ft_flowtree_flows": ([p, p, p, p, i64, p, p, i64, p, p, p, p, p, p, p], ctypes.c_int),
        "ft_quadtree_pairs": ([p, p, p, p, i64, p, p, i64, p, p], ctypes.c_int),
        "ft_act_knn": ([p, p, p, p, i64, p, i32, i32, i32, p, p, p], ctypes.c_int),
        "ft_act_pairs": ([p, p, p, p, i64, p, p, i64, i32, p, p], ctypes.c_int),
        "ft_last_rerank_stats": ([p, p], ctypes.c_int),
        "ft_last_quadtree_stats": ([p, p], ctypes.c_int),
        "ft_quadtree_eps_pairs": ([p, p, p, p, i64, p, p, i64, ctypes.c_double, p, p], ctypes.c_int),
        "ft_quadtree_eps_knn": ([p, p, p, p, i64, p, i32, ctypes.c_double, i32, p, p, p], ctypes.c_int),
        "ft_exact_knn": ([p, p, p, p, i64, p, i32, i32, p, p, p], ctypes.c_int),
        "ft_exact_pairs": ([p, p, p, p, i64, p, p, i64, p, p], ctypes.c_int),
        "ft_sinkhorn_knn": ([p, p, p, p, i64, p, i32, i32, ctypes.c_float, i32, p, p, p], ctypes.c_int),
        "ft_sinkhorn_pairs": ([p, p, p, p, i64, p, p, i64, i32, ctypes.c_float, p, p], ctypes.c_int),
        "ft_set_autotune": ([p, i32], ctypes.c_int),
        "ft_last_batched_stats": ([p, p, p, i32], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _LIB = lib
    return lib


def _check(rc: int):
    if rc != 0:
        raise FtError(rc, load().ft_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _u32(t):
    """uint32 data as an int32 CUDA tensor (same bits)."""
    if t.dtype == torch.int32:
        return t.contiguous()
    if t.dtype == torch.uint32:
        return t.contiguous().view(torch.int32)
    return t.to(torch.int64).to(torch.int32).contiguous()


def _i64(t):
    return t.to(torch.int64).contiguous()


class Index:
    """A built quadtree over X plus the packed dataset (ft_build_tree)."""

    def __init__(self, handle, V, d, n_docs):
        self._h = handle
        self.V, self.d, self.n_docs = V, d, n_docs

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _LIB is not None:
            _LIB.ft_free(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        buf = (ctypes.c_int64 * 8)()
        _check(load().ft_index_info(self._h, ctypes.cast(buf, ctypes.c_void_p)))
        keys = ["V", "d", "B", "Q", "n_docs", "height", "n_nodes", "max_doc_size"]
        return dict(zip(keys, list(buf)))

    def export_tree(self):
        """(perm, adj_lcp, leaf_depth) as CUDA tensors (int32 / uint8)."""
        dev = torch.device("cuda", torch.cuda.current_device())
        perm = torch.empty(self.V, dtype=torch.int32, device=dev)
        lcp = torch.empty(self.V, dtype=torch.uint8, device=dev)
        ld = torch.empty(self.V, dtype=torch.uint8, device=dev)
        _check(load().ft_export_tree(self._h, _ptr(perm), _ptr(lcp), _ptr(ld), _stream()))
        return perm, lcp, ld

    def set_autotune(self, level: int):
        _check(load().ft_set_autotune(self._h, level))

    def last_batched_stats(self):
        ms = ctypes.c_double(0.0)
        buf = ctypes.create_string_buffer(256)
        _check(load().ft_last_batched_stats(self._h, ctypes.byref(ms), buf, 256))
        return ms.value, buf.value.decode()

    def last_pipeline_stats(self):
        """(prune ms, rerank ms) of the last knn_pipeline call (HIP events)."""
        a, b = ctypes.c_double(0.0), ctypes.c_double(0.0)
        _check(load().ft_last_pipeline_stats(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def last_select_exact_rows(self):
        """Rows of the last quadtree_knn call whose sampled one-pass select
        fell back to the exact select."""
        n = ctypes.c_int64(0)
        _check(load().ft_last_quadtree_stats(self._h, ctypes.byref(n)))
        return n.value

    def last_rerank_ms(self):
        """Device time of the estimate kernels of the last act_knn or
        sinkhorn_knn call."""
        ms = ctypes.c_double(0.0)
        _check(load().ft_last_rerank_stats(self._h, ctypes.byref(ms)))
        return ms.value


def build_tree(X, shift, B, doc_off, doc_id, doc_mass, Q) -> Index:
    """ft_build_tree: X (V x d float32 CUDA), shift (d ints, host), doc CSR."""
    X = X.to(torch.float32).contiguous()
    V, d = X.shape
    sh = (ctypes.c_int64 * d)(*[int(v) for v in shift])
    doc_off = _i64(doc_off)
    doc_id, doc_mass = _u32(doc_id), _u32(doc_mass)
    h = ctypes.c_void_p()
    _check(load().ft_build_tree(_ptr(X), V, d, ctypes.cast(sh, ctypes.c_void_p), B, _ptr(doc_off),
                                _ptr(doc_id), _ptr(doc_mass), doc_off.numel() - 1, Q, _stream(),
                                ctypes.byref(h)))
    ix = Index(h, V, d, doc_off.numel() - 1)
    ix.doc_sizes = doc_off[1:] - doc_off[:-1]
    ix.doc_nnz = doc_id.numel()
    ix.doc_mass = doc_mass.clone()  # the weights autograd.FlowtreeCost checks d_w against
    ix.Q = Q
    return ix


def _queries(q_off, q_id, q_mass):
    return _i64(q_off), _u32(q_id), _u32(q_mass)


def quadtree_knn(index: Index, q_off, q_id, q_mass, k: int, cand=None):
    """ft_quadtree_knn -> (keys int64 [n_q, k] (uint64 bits), docs int64 [n_q, k])."""
    q_off, q_id, q_mass = _queries(q_off, q_id, q_mass)
    n_q = q_off.numel() - 1
    dev = q_off.device
    cand_t = _i64(cand) if cand is not None else None
    n_cand = cand_t.shape[-1] if cand_t is not None else 0
    keys = torch.empty((n_q, k), dtype=torch.int64, device=dev)
    docs = torch.empty((n_q, k), dtype=torch.int64, device=dev)
    _check(load().ft_quadtree_knn(index.handle, _ptr(q_off), _ptr(q_id), _ptr(q_mass), n_q,
                                  _ptr(cand_t), n_cand, k, _ptr(keys), _ptr(docs), _stream()))
    return keys, docs


def flowtree_knn(index: Index, q_off, q_id, q_mass, k: int, cand=None, mode: int = FT_BATCHED):
    """ft_flowtree_knn -> (costs float32 [n_q, k], docs int64 [n_q, k])."""
    q_off, q_id, q_mass = _queries(q_off, q_id, q_mass)
    n_q = q_off.numel() - 1
    dev = q_off.device
    cand_t = _i64(cand) if cand is not None else None
    n_cand = cand_t.shape[-1] if cand_t is not None else 0
    costs = torch.empty((n_q, k), dtype=torch.float32, device=dev)
    docs = torch.empty((n_q, k), dtype=torch.int64, device=dev)
    _check(load().ft_flowtree_knn(index.handle, _ptr(q_off), _ptr(q_id), _ptr(q_mass), n_q,
                                  _ptr(cand_t), n_cand, k, mode, _ptr(costs), _ptr(docs), _stream()))
    return costs, docs


def knn_pipeline(index: Index, q_off, q_id, q_mass, prune_k: int, k: int):
    """ft_knn_pipeline -> (costs float32 [n_q, k], docs int64 [n_q, k]): the
    Quadtree prune of every doc to prune_k, then the batched Flowtree rerank
    to k, in one call."""
    q_off, q_id, q_mass = _queries(q_off, q_id, q_mass)
    n_q = q_off.numel() - 1
    costs = torch.empty((n_q, k), dtype=torch.float32, device=q_off.device)
    docs = torch.empty((n_q, k), dtype=torch.int64, device=q_off.device)
    _check(load().ft_knn_pipeline(index.handle, _ptr(q_off), _ptr(q_id), _ptr(q_mass), n_q, prune_k, k,
                                  _ptr(costs), _ptr(docs), _stream()))
    return costs, docs


def flowtree_knn_noalloc(index: Index, q_off, q_id, q_mass, k: int, cand, out=None):
    """ft_flowtree_knn_noalloc -> (costs float32 [n_q, k], docs int64 [n_q, k]).
    The library allocates nothing; pass out=(costs, docs) to reuse output
    tensors as well."""
    q_off, q_id, q_mass = _queries(q_off, q_id, q_mass)
    n_q = q_off.numel() - 1
    cand_t = _i64(cand)
    n_cand = cand_t.shape[-1]
    if out is None:
        costs = torch.empty((n_q, k), dtype=torch.float32, device=q_off.device)
        docs = torch.empty((n_q, k), dtype=torch.int64, device=q_off.device)
    else:
        costs, docs = out
    _check(load().ft_flowtree_knn_noalloc(index.handle, _ptr(q_off), _ptr(q_id), _ptr(q_mass), n_q,
                                          _ptr(cand_t), n_cand, k, _ptr(costs), _ptr(docs), _stream()))
    return costs, docs


def act_knn(index: Index, q_off, q_id, q_mass, k: int, iters: int = 1, cand=None):
    """ft_act_knn -> (costs float32 [n_q, k], docs int64 [n_q, k]); iters = 0
    is Relaxed WMD."""
    q_off, q_id, q_mass = _queries(q_off, q_id, q_mass)
    n_q = q_off.numel() - 1
    dev = q_off.device
    cand_t = _i64(cand) if cand is not None else None
    n_cand = cand_t.shape[-1] if cand_t is not None else 0
    costs = torch.empty((n_q, k), dtype=torch.float32, device=dev)
    docs = torch.empty((n_q, k), dtype=torch.int64, device=dev)
    _check(load().ft_act_knn(index.handle, _ptr(q_off), _ptr(q_id), _ptr(q_mass), n_q,
                             _ptr(cand_t), n_cand, iters, k, _ptr(costs), _ptr(docs), _stream()))
    return costs, docs


def act_pairs(index: Index, q_off, q_id, q_mass, pair_q, pair_d, iters: int = 1):
    """ft_act_pairs -> float32 ACT-iters value per pair."""
    q_off, q_id, q_mass = _queries(q_off, q_id, q_mass)
    pair_q, pair_d = _i64(pair_q), _i64(pair_d)
    out = torch.empty(pair_q.numel(), dtype=torch.float32, device=q_off.device)
    _check(load().ft_act_pairs(index.handle, _ptr(q_off), _ptr(q_id), _ptr(q_mass),
                               q_off.numel() - 1, _ptr(pair_q), _ptr(pair_d), pair_q.numel(), iters,
                               _ptr(out), _stream()))
    return out


def sinkhorn_knn(index: Index, q_off, q_id, q_mass, k: int, iters: int = 1, eta: float = 30.0, cand=None):
    """ft_sinkhorn_knn -> (costs float32 [n_q, k], docs int64 [n_q, k])."""
    q_off, q_id, q_mass = _queries(q_off, q_id, q_mass)
    n_q = q_off.numel() - 1
    dev = q_off.device
    cand_t = _i64(cand) if cand is not None else None
    n_cand = cand_t.shape[-1] if cand_t is not None else 0
    costs = torch.empty((n_q, k), dtype=torch.float32, device=dev)
    docs = torch.empty((n_q, k), dtype=torch.int64, device=dev)
    _check(load().ft_sinkhorn_knn(index.handle, _ptr(q_off), _ptr(q_id), _ptr(q_mass), n_q,
                                  _ptr(cand_t), n_cand, iters, eta, k, _ptr(costs), _ptr(docs), _stream()))
    return costs, docs


def sinkhorn_pairs(index: Index, q_off, q_id, q_mass, pair_q, pair_d, iters: int = 1, eta: float = 30.0):
    """ft_sinkhorn_pairs -> float32 Sinkhorn value per pair."""
    q_off, q_id, q_mass = _queries(q_off, q_id, q_mass)
    pair_q, pair_d = _i64(pair_q), _i64(pair_d)
    out = torch.empty(pair_q.numel(), dtype=torch.float32, device=q_off.device)
    _check(load().ft_sinkhorn_pairs(index.handle, _ptr(q_off), _ptr(q_id), _ptr(q_mass),
                                    q_off.numel() - 1, _ptr(pair_q), _ptr(pair_d), pair_q.numel(), iters, eta,
                                    _ptr(out), _stream()))
    return out


def exact_knn(index: Index, q_off, q_id, q_mass, k: int, cand=None):
    """ft_exact_knn -> (W1 float32 [n_q, k], docs int64 [n_q, k])."""
    q_off, q_id, q_mass = _queries(q_off, q_id, q_mass)
    n_q = q_off.numel() - 1
    dev = q_off.device
    cand_t = _i64(cand) if cand is not None else None
    n_cand = cand_t.shape[-1] if cand_t is not None else 0
    costs = torch.empty((n_q, k), dtype=torch.float32, device=dev)
    docs = torch.empty((n_q, k), dtype=torch.int64, device=dev)
    _check(load().ft_exact_knn(index.handle, _ptr(q_off), _ptr(q_id), _ptr(q_mass), n_q,
                               _ptr(cand_t), n_cand, k, _ptr(costs), _ptr(docs), _stream()))
    return costs, docs


def exact_pairs(index: Index, q_off, q_id, q_mass, pair_q, pair_d):
    """ft_exact_pairs -> float32 exact W1 per pair."""
    q_off, q_id, q_mass = _queries(q_off, q_id, q_mass)
    pair_q, pair_d = _i64(pair_q), _i64(pair_d)
    out = torch.empty(pair_q.numel(), dtype=torch.float32, device=q_off.device)
    _check(load().ft_exact_pairs(index.handle, _ptr(q_off), _ptr(q_id), _ptr(q_mass),
                                 q_off.numel() - 1, _ptr(pair_q), _ptr(pair_d), pair_q.numel(), _ptr(out),
                                 _stream()))
    return out


def quadtree_eps_pairs(index: Index, q_off, q_id, q_mass, pair_q, pair_d, eps: float):
    """ft_quadtree_eps_pairs -> float64 eps-weighted Quadtree value per pair."""
    q_off, q_id, q_mass = _queries(q_off, q_id, q_mass)
    pair_q, pair_d = _i64(pair_q), _i64(pair_d)
    out = torch.empty(pair_q.numel(), dtype=torch.float64, device=q_off.device)
    _check(load().ft_quadtree_eps_pairs(index.handle, _ptr(q_off), _ptr(q_id), _ptr(q_mass),
                                        q_off.numel() - 1, _ptr(pair_q), _ptr(pair_d), pair_q.numel(), eps,
                                        _ptr(out), _stream()))
    return out


def quadtree_eps_knn(index: Index, q_off, q_id, q_mass, k: int, cand, eps: float):
    """ft_quadtree_eps_knn -> (values float32 [n_q, k], docs int64 [n_q, k])."""
    q_off, q_id, q_mass = _queries(q_off, q_id, q_mass)
    n_q = q_off.numel() - 1
    cand_t = _i64(cand)
    costs = torch.empty((n_q, k), dtype=torch.float32, device=q_off.device)
    docs = torch.empty((n_q, k), dtype=torch.int64, device=q_off.device)
    _check(load().ft_quadtree_eps_knn(index.handle, _ptr(q_off), _ptr(q_id), _ptr(q_mass), n_q,
                                      _ptr(cand_t), cand_t.shape[-1], eps, k, _ptr(costs), _ptr(docs),
                                      _stream()))
    return costs, docs


def quadtree_pairs(index: Index, q_off, q_id, q_mass, pair_q, pair_d):
    """ft_quadtree_pairs -> int64 keys (uint64 bits) per pair."""
    q_off, q_id, q_mass = _queries(q_off, q_id, q_mass)
    pair_q, pair_d = _i64(pair_q), _i64(pair_d)
    out = torch.empty(pair_q.numel(), dtype=torch.int64, device=q_off.device)
    _check(load().ft_quadtree_pairs(index.handle, _ptr(q_off), _ptr(q_id), _ptr(q_mass),
                                    q_off.numel() - 1, _ptr(pair_q), _ptr(pair_d), pair_q.numel(),
                                    _ptr(out), _stream()))
    return out


def flowtree_flows(index: Index, q_off, q_id, q_mass, pair_q, pair_d):
    """ft_flowtree_flows -> list of (doc point, query point, eta, bind) int64
    arrays per pair (host numpy), in the library's emission order."""
    q_off, q_id, q_mass = _queries(q_off, q_id, q_mass)
    pair_q, pair_d = _i64(pair_q), _i64(pair_d)
    n = pair_q.numel()
    sizes = (q_off[pair_q + 1] - q_off[pair_q]) + index.doc_sizes[pair_d]
    cap = torch.zeros(n + 1, dtype=torch.int64, device=q_off.device)
    cap[1:] = torch.cumsum(sizes, 0)
    total = int(cap[-1].item())
    dev = q_off.device
    cnt = torch.empty(n, dtype=torch.int32, device=dev)
    fd = torch.empty(total, dtype=torch.int32, device=dev)
    fq = torch.empty(total, dtype=torch.int32, device=dev)
    fe = torch.empty(total, dtype=torch.int32, device=dev)
    fb = torch.empty(total, dtype=torch.uint8, device=dev)
    _check(load().ft_flowtree_flows(index.handle, _ptr(q_off), _ptr(q_id), _ptr(q_mass),
                                    q_off.numel() - 1, _ptr(pair_q), _ptr(pair_d), n, _ptr(cap),
                                    _ptr(cnt), _ptr(fd), _ptr(fq), _ptr(fe), _ptr(fb), _stream()))
    cap_h, cnt_h = cap.cpu().numpy(), cnt.cpu().numpy()
    fd_h = fd.cpu().numpy().view("uint32").astype("int64")
    fq_h = fq.cpu().numpy().view("uint32").astype("int64")
    fe_h = fe.cpu().numpy().view("uint32").astype("int64")
    fb_h = fb.cpu().numpy().astype("int64")
    out = []
    for p in range(n):
        a, c = cap_h[p], cnt_h[p]
        out.append((fd_h[a:a + c], fq_h[a:a + c], fe_h[a:a + c], fb_h[a:a + c]))
    return out


def flowtree_cost_grad(index: Index, X, q_off, q_id, q_mass, pair_q, pair_d, mode: int,
                       grad_out=None, cost=None, grad_X=None, grad_qmass=None, grad_dmass=None):
    """ft_flowtree_cost_grad (FT_FWD writes cost; FT_BWD adds gradients)."""
    q_off, q_id, q_mass = _queries(q_off, q_id, q_mass)
    pair_q, pair_d = _i64(pair_q), _i64(pair_d)
    X = X.contiguous()
    _check(load().ft_flowtree_cost_grad(index.handle, _ptr(X), _ptr(q_off), _ptr(q_id), _ptr(q_mass),
                                        q_off.numel() - 1, _ptr(pair_q), _ptr(pair_d), pair_q.numel(),
                                        mode, _ptr(grad_out), _ptr(cost), _ptr(grad_X),
                                        _ptr(grad_qmass), _ptr(grad_dmass), _stream()))
