"""CPU oracle for the Quadtree / Flowtree hot path (arXiv 1910.04126).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import this
package.  It shares no code with the GPU library; both sides start from the
same seeded inputs produced by ``gen``.

Contents, each following the paper:

* ``Tree``: the randomly shifted quadtree (Section 2), built by literal
  recursive halving in ``oracle.c``; Morton rank = depth-first leaf order.
* ``Tree.quadtree``: closed form sum_v w(v) |mu(v) - nu(v)| (Section 2).
* ``Tree.quadtree_eps``: the same with edge weights (2^level)^(1 - eps), the
  tree of the proof of the uniform-distribution Flowtree upper bound.
* ``Tree.flowtree``: bottom-up greedy tree flow (Appendix A.1) priced with
  Euclidean distances (Section 3), float64.
* ``exact_w1_*``: W1 of Section 1, eq. (1), three independent ways (LP,
  successive shortest paths, permutations) for tiny inputs.
* ``tree_w1_lp`` / ``flow_face_bracket``: the tree-metric transport LP and
  the min / max Euclidean price over its optimal face (tiny inputs).
* ``frozen_cost`` / ``frozen_grad``: Flowtree cost and its gradient with the
  tree and the flow pattern held fixed (the paper gives no gradient; the
  reading is documented with the functions).
* ``topk``: k smallest by (key, doc id).
* ``rwmd`` / ``act``: the quadratic-time comparison estimates that follow
  Flowtree in the paper's pipelines -- Relaxed WMD (Section 1.1) and the
  Approximate Constrained Transfers with i iterations (Section 4.1), float64.
* ``sinkhorn``: Sinkhorn with a fixed small number of iterations (Section
  4.1, regularisation of Appendix "Sinkhorn regularization parameter"),
  float64.

Parity of the GPU path is checked against these functions.  Functions with no
independent pin are marked "parity unpinned" in their docstring.
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None
_LOCK = threading.Lock()

OR_OK, OR_EINVAL, OR_ENOMEM = 0, -1, -2


class OracleError(RuntimeError):
    pass


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (IEEE float64, no contraction); return path."""
    src = os.path.join(_HERE, "oracle.c")
    out = os.path.join(_HERE, "liboracle.so")
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-shared", "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


def load(path: str):
    """Load an oracle library (the default one, or a variant built elsewhere
    from a modified copy of oracle.c -- used by the mutation tests)."""
    lib = ctypes.CDLL(path)
    p, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.oracle_tree_build.argtypes = [p, i64, i32, p, i32, ctypes.POINTER(p)]
    lib.oracle_tree_build.restype = ctypes.c_int
    lib.oracle_tree_free.argtypes = [p]
    lib.oracle_tree_free.restype = None
    lib.oracle_tree_nodes.argtypes = [p]
    lib.oracle_tree_nodes.restype = i64
    lib.oracle_tree_phi.argtypes = [p]
    lib.oracle_tree_phi.restype = ctypes.c_double
    lib.oracle_tree_export.argtypes = [p] * 8
    lib.oracle_tree_export.restype = None
    lib.oracle_tree_dist.argtypes = [p, i64, i64]
    lib.oracle_tree_dist.restype = ctypes.c_uint64
    lib.oracle_lca_depth.argtypes = [p, i64, i64]
    lib.oracle_lca_depth.restype = i32
    lib.oracle_quadtree.argtypes = [p, p, p, i64, p, p, i64, i32, p]
    lib.oracle_quadtree.restype = ctypes.c_int
    lib.oracle_quadtree_eps.argtypes = [p, p, p, i64, p, p, i64, i32, ctypes.c_double, p]
    lib.oracle_quadtree_eps.restype = ctypes.c_int
    lib.oracle_flowtree.argtypes = [p, p, p, p, i64, p, p, i64, i32, p, p, p, p, p, p]
    lib.oracle_flowtree.restype = ctypes.c_int
    lib.oracle_exact_w1_ssp.argtypes = [p, i32, p, p, i64, p, p, i64, i32, p]
    lib.oracle_exact_w1_ssp.restype = ctypes.c_int
    lib.oracle_quadtree_pairs.argtypes = [p] * 9 + [i64, i32, p]
    lib.oracle_quadtree_pairs.restype = ctypes.c_int
    lib.oracle_flowtree_pairs.argtypes = [p] * 10 + [i64, i32, p]
    lib.oracle_flowtree_pairs.restype = ctypes.c_int
    return lib


def _lib():
    global _LIB
    with _LOCK:
        if _LIB is None:
            _LIB = load(build())
    return _LIB


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


class Tree:
    """Randomly shifted quadtree over X (Section 2); see oracle.c for the
    reading of the grid, the leaves and the child order."""

    def __init__(self, X: np.ndarray, shift: np.ndarray, B: int = 30, lib=None):
        self._L = lib if lib is not None else _lib()
        self.X = np.ascontiguousarray(X, dtype=np.float32)
        self.V, self.d = self.X.shape
        self.B = int(B)
        self.shift = _i64(shift)
        h = ctypes.c_void_p()
        rc = self._L.oracle_tree_build(_p(self.X), self.V, self.d, _p(self.shift), self.B,
                                      ctypes.byref(h))
        if rc != OR_OK:
            raise OracleError("tree build failed (%d)" % rc)
        self._h = h
        self.n_nodes = int(self._L.oracle_tree_nodes(h))
        self.phi = float(self._L.oracle_tree_phi(h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None:
            self._L.oracle_tree_free(h)
            self._h = None

    # ---- structure -----------------------------------------------------
    def export(self) -> dict:
        V, n = self.V, self.n_nodes
        out = dict(code=np.empty((V, self.d), np.uint32), rank_of=np.empty(V, np.int64),
                   leaf_depth=np.empty(V, np.int32), node_depth=np.empty(n, np.int32),
                   node_parent=np.empty(n, np.int64), node_first=np.empty(n, np.int64),
                   node_last=np.empty(n, np.int64))
        self._L.oracle_tree_export(self._h, *[_p(out[k]) for k in
                                             ("code", "rank_of", "leaf_depth", "node_depth",
                                              "node_parent", "node_first", "node_last")])
        return out

    def tree_dist(self, x: int, y: int) -> int:
        """t(x, y) in grid units (Section 2)."""
        return int(self._L.oracle_tree_dist(self._h, int(x), int(y)))

    def lca_depth(self, x: int, y: int) -> int:
        return int(self._L.oracle_lca_depth(self._h, int(x), int(y)))

    def grid_unit(self) -> float:
        """Length of one grid unit: 2*Phi / 2**B."""
        return 2.0 * self.phi / float(1 << self.B)

    # ---- estimators ------------------------------------------------------
    def quadtree(self, mu_id, mu_m, nu_id, nu_m, Q: int) -> int:
        """Quadtree estimate U = sum_{v != root} 2^(B-depth v) |mu(v) - nu(v)|
        as an exact integer in units of 2^-Q mass x grid unit (Section 2)."""
        mu_id, mu_m, nu_id, nu_m = _u32(mu_id), _u32(mu_m), _u32(nu_id), _u32(nu_m)
        out = np.zeros(1, np.uint64)
        rc = self._L.oracle_quadtree(self._h, _p(mu_id), _p(mu_m), len(mu_id), _p(nu_id),
                                    _p(nu_m), len(nu_id), Q, _p(out))
        if rc != OR_OK:
            raise OracleError("quadtree: invalid input (%d)" % rc)
        return int(out[0])

    def quadtree_eps(self, mu_id, mu_m, nu_id, nu_m, Q: int, eps: float) -> float:
        """Quadtree with eps-weighted edges: sum over non-root cells v of
        (2^(B-depth v))^(1-eps) |mu(v) - nu(v)|, masses as fractions, float64
        (the weights of the proof of the uniform-distribution Flowtree bound;
        eps = 0 is the plain Quadtree / 2^Q)."""
        mu_id, mu_m, nu_id, nu_m = _u32(mu_id), _u32(mu_m), _u32(nu_id), _u32(nu_m)
        out = ctypes.c_double(0.0)
        rc = self._L.oracle_quadtree_eps(self._h, _p(mu_id), _p(mu_m), len(mu_id), _p(nu_id),
                                        _p(nu_m), len(nu_id), Q, ctypes.c_double(eps), ctypes.byref(out))
        if rc != OR_OK:
            raise OracleError("quadtree_eps: invalid input (%d)" % rc)
        return out.value

    def quadtree_value(self, *a, Q: int) -> float:
        """Quadtree estimate in the units of X (float64)."""
        return self.quadtree(*a, Q=Q) * self.grid_unit() / float(1 << Q)

    def flowtree(self, mu_id, mu_m, nu_id, nu_m, Q: int, with_cost: bool = True):
        """Flowtree (Appendix A.1 greedy, Section 3 price).

        mu is the dataset distribution, nu the query.  Returns (cost, flows)
        where flows is a dict of arrays in emission order: ``mu`` / ``nu``
        (indices into the support arrays), ``eta`` (integer mass), ``bind``
        (0: the match used up the mu-item, 1: the nu-item, 2: both).
        cost = 2^-Q sum eta ||x - y||_2 in float64.
        """
        mu_id, mu_m, nu_id, nu_m = _u32(mu_id), _u32(mu_m), _u32(nu_id), _u32(nu_m)
        cap = len(mu_id) + len(nu_id) + 1
        a = np.empty(cap, np.int32)
        b = np.empty(cap, np.int32)
        eta = np.empty(cap, np.uint32)
        bind = np.empty(cap, np.int8)
        ne = ctypes.c_int64(0)
        cost = ctypes.c_double(0.0)
        rc = self._L.oracle_flowtree(self._h, _p(self.X) if with_cost else None, _p(mu_id),
                                    _p(mu_m), len(mu_id), _p(nu_id), _p(nu_m), len(nu_id), Q,
                                    _p(a), _p(b), _p(eta), _p(bind), ctypes.byref(ne),
                                    ctypes.byref(cost))
        if rc != OR_OK:
            raise OracleError("flowtree: invalid input (%d)" % rc)
        n = ne.value
        flows = dict(mu=a[:n].copy(), nu=b[:n].copy(), eta=eta[:n].copy(), bind=bind[:n].copy())
        return cost.value, flows

    # ---- batches (CSR inputs) ------------------------------------------
    def quadtree_pairs(self, q_off, q_id, q_m, d_off, d_id, d_m, pair_q, pair_d, Q):
        arrs = [_i64(q_off), _u32(q_id), _u32(q_m), _i64(d_off), _u32(d_id), _u32(d_m),
                _i64(pair_q), _i64(pair_d)]
        out = np.empty(len(arrs[6]), np.uint64)
        rc = self._L.oracle_quadtree_pairs(self._h, *[_p(a) for a in arrs], len(arrs[6]), Q,
                                          _p(out))
        if rc != OR_OK:
            raise OracleError("quadtree_pairs: invalid input (%d)" % rc)
        return out

    def flowtree_pairs(self, q_off, q_id, q_m, d_off, d_id, d_m, pair_q, pair_d, Q):
        arrs = [_i64(q_off), _u32(q_id), _u32(q_m), _i64(d_off), _u32(d_id), _u32(d_m),
                _i64(pair_q), _i64(pair_d)]
        out = np.empty(len(arrs[6]), np.float64)
        rc = self._L.oracle_flowtree_pairs(self._h, _p(self.X), *[_p(a) for a in arrs],
                                          len(arrs[6]), Q, _p(out))
        if rc != OR_OK:
            raise OracleError("flowtree_pairs: invalid input (%d)" % rc)
        return out


# --------------------------------------------------------------------------
# k nearest neighbours (Section 1 problem statement)
# --------------------------------------------------------------------------

def topk(keys: np.ndarray, ids: np.ndarray, k: int):
    """The k smallest entries ordered by (key, id); returns (keys, ids)."""
    order = np.lexsort((np.asarray(ids), np.asarray(keys)))[:k]
    return np.asarray(keys)[order], np.asarray(ids)[order]


# --------------------------------------------------------------------------
# Exact W1 (Section 1, eq. 1) -- tiny inputs only
# --------------------------------------------------------------------------

def _dist_matrix(X, a_id, b_id):
    A = np.asarray(X, np.float64)[np.asarray(a_id, np.int64)]
    Bm = np.asarray(X, np.float64)[np.asarray(b_id, np.int64)]
    diff = A[:, None, :] - Bm[None, :, :]
    return np.sqrt((diff * diff).sum(-1))


def exact_w1_lp(X, mu_id, mu_m, nu_id, nu_m, Q: int = None, cost=None) -> float:
    """W1 as the transportation LP over couplings with marginals mu, nu
    (scipy HiGHS), Euclidean cost unless ``cost`` is given.  Masses are
    integers scaled by 2^-Q, or float weights when Q is None."""
    from scipy.optimize import linprog
    C = _dist_matrix(X, mu_id, nu_id) if cost is None else np.asarray(cost, np.float64)
    scale = 1.0 if Q is None else float(1 << Q)
    a = np.asarray(mu_m, np.float64) / scale
    b = np.asarray(nu_m, np.float64) / scale
    n, m = C.shape
    A = np.zeros((n + m, n * m))
    for i in range(n):
        A[i, i * m:(i + 1) * m] = 1.0
    for j in range(m):
        A[n + j, j::m] = 1.0
    res = linprog(C.ravel(), A_eq=A, b_eq=np.concatenate([a, b]), bounds=(0, None),
                  method="highs")
    if res.status != 0:
        raise OracleError("LP failed: %s" % res.message)
    return float(res.fun)


def exact_w1_ssp(X, mu_id, mu_m, nu_id, nu_m, Q: int) -> float:
    """W1 by successive shortest paths on integer masses (oracle.c)."""
    X = np.ascontiguousarray(X, np.float32)
    mu_id, mu_m, nu_id, nu_m = _u32(mu_id), _u32(mu_m), _u32(nu_id), _u32(nu_m)
    out = ctypes.c_double(0.0)
    rc = _lib().oracle_exact_w1_ssp(_p(X), X.shape[1], _p(mu_id), _p(mu_m), len(mu_id),
                                    _p(nu_id), _p(nu_m), len(nu_id), Q, ctypes.byref(out))
    if rc != OR_OK:
        raise OracleError("ssp failed (%d)" % rc)
    return out.value


def exact_w1_brute(X, mu_id, nu_id) -> float:
    """W1 between two uniform distributions of equal support size s <= 7:
    by Birkhoff's theorem an optimal coupling is a permutation matrix / s."""
    C = _dist_matrix(X, mu_id, nu_id)
    s = C.shape[0]
    if C.shape[1] != s or s > 7:
        raise ValueError("brute force needs equal sizes <= 7")
    best = min(sum(C[i, p[i]] for i in range(s)) for p in itertools.permutations(range(s)))
    return best / s


def tree_dist_matrix(tree: Tree, mu_id, nu_id) -> np.ndarray:
    return np.array([[tree.tree_dist(x, y) for y in nu_id] for x in mu_id], dtype=np.float64)


def tree_w1_lp(tree: Tree, mu_id, mu_m, nu_id, nu_m, Q: int) -> float:
    """Optimal transport cost under the tree metric t (grid units x 2^-Q mass
    fractions), solved as an LP -- the quantity the Quadtree closed form
    equals (Section 2)."""
    T = tree_dist_matrix(tree, mu_id, nu_id)
    return exact_w1_lp(tree.X, mu_id, mu_m, nu_id, nu_m, Q, cost=T)


def flow_face_bracket(tree: Tree, mu_id, mu_m, nu_id, nu_m, Q: int):
    """(min, max) of sum f ||x - y|| over the couplings f that are optimal for
    the tree metric.  Any tree-optimal flow -- whatever order the greedy
    matches in -- prices inside this bracket (Section 3 definition of
    Flowtree as the Euclidean price of a tree-optimal flow)."""
    from scipy.optimize import linprog
    T = tree_dist_matrix(tree, mu_id, nu_id)
    C = _dist_matrix(tree.X, mu_id, nu_id)
    a = np.asarray(mu_m, np.float64) / float(1 << Q)
    b = np.asarray(nu_m, np.float64) / float(1 << Q)
    n, m = C.shape
    A = np.zeros((n + m, n * m))
    for i in range(n):
        A[i, i * m:(i + 1) * m] = 1.0
    for j in range(m):
        A[n + j, j::m] = 1.0
    beq = np.concatenate([a, b])
    U = tree.quadtree(mu_id, mu_m, nu_id, nu_m, Q) / float(1 << Q)
    slack = 1e-9 * max(1.0, U)
    out = []
    for sgn in (1.0, -1.0):
        res = linprog(sgn * C.ravel(), A_ub=T.ravel()[None, :], b_ub=[U + slack], A_eq=A,
                      b_eq=beq, bounds=(0, None), method="highs")
        if res.status != 0:
            raise OracleError("bracket LP failed: %s" % res.message)
        out.append(sgn * res.fun)
    return out[0], out[1]


# --------------------------------------------------------------------------
# Gradient with the tree and the flow pattern frozen
# --------------------------------------------------------------------------

def frozen_cost(X, mu_id, nu_id, flows, mu_w, nu_w) -> float:
    """Flowtree cost with the emission pattern of ``flows`` frozen.

    Reading (the paper defines no gradient): every emission e transports the
    current unmatched mass of the item it used up (its "bind" item; the mu
    item when both were used up), so eta_e is a linear function of the
    continuous weights mu_w, nu_w (mass / 2^Q):
        eta_e = r[bind_e];  r[mu_e] -= eta_e;  r[nu_e] -= eta_e.
    C = sum_e eta_e * ||x_mu_e - x_nu_e||_2, float64.
    """
    X = np.asarray(X, np.float64)
    rm = np.array(mu_w, np.float64)
    rn = np.array(nu_w, np.float64)
    c = 0.0
    for a, b, bind in zip(flows["mu"], flows["nu"], flows["bind"]):
        eta = rn[b] if bind == 1 else rm[a]
        rm[a] -= eta
        rn[b] -= eta
        c += eta * np.linalg.norm(X[mu_id[a]] - X[nu_id[b]])
    return float(c)


def frozen_grad(X, mu_id, nu_id, flows, mu_w, nu_w):
    """Gradient of ``frozen_cost`` w.r.t. X (V x d), mu_w and nu_w.

    Coordinates: d/dx of eta_e ||x_a - x_b|| is eta_e (x_a - x_b) / D_e on a
    and the negative on b, 0 when D_e = 0.  Weights by reverse accumulation:
    lambda_e = D_e - acc[mu_e] - acc[nu_e]; acc[bind_e] += lambda_e, for e
    from last to first; then d/dmu_w = acc over mu items, d/dnu_w likewise.
    """
    X = np.asarray(X, np.float64)
    rm = np.array(mu_w, np.float64)
    rn = np.array(nu_w, np.float64)
    E = len(flows["mu"])
    eta = np.empty(E)
    D = np.empty(E)
    for e, (a, b, bind) in enumerate(zip(flows["mu"], flows["nu"], flows["bind"])):
        eta[e] = rn[b] if bind == 1 else rm[a]
        rm[a] -= eta[e]
        rn[b] -= eta[e]
        D[e] = np.linalg.norm(X[mu_id[a]] - X[nu_id[b]])
    gX = np.zeros_like(X)
    for e in range(E):
        if D[e] > 0:
            a, b = int(flows["mu"][e]), int(flows["nu"][e])
            g = eta[e] * (X[mu_id[a]] - X[nu_id[b]]) / D[e]
            gX[mu_id[a]] += g
            gX[nu_id[b]] -= g
    acc_m = np.zeros(len(mu_w))
    acc_n = np.zeros(len(nu_w))
    for e in range(E - 1, -1, -1):
        a, b, bind = int(flows["mu"][e]), int(flows["nu"][e]), int(flows["bind"][e])
        lam = D[e] - acc_m[a] - acc_n[b]
        if bind == 1:
            acc_n[b] += lam
        else:
            acc_m[a] += lam
    return gX, acc_m, acc_n


# --------------------------------------------------------------------------
# Relaxed WMD and ACT-i (Section 1.1 "prior work", Section 4.1 baselines)
# --------------------------------------------------------------------------

def _act_one_way(C, a, b, iters: int) -> float:
    """One direction of ACT-iters with integer masses a (sources, rows of C)
    and b (targets, columns).  Each source takes its targets by ascending
    distance (equal distances by target index); the first ``iters`` of them
    each receive at most their own mass b_j, and what is left goes to the
    next nearest target with no limit.  iters = 0 sends everything to the
    nearest target (one side of R-WMD).  Returns sum of mass x distance in
    mass units (not yet divided by 2^Q)."""
    total = 0.0
    m = C.shape[1]
    for i in range(C.shape[0]):
        order = np.argsort(C[i], kind="stable")
        r = int(a[i])
        for t in range(min(iters, m)):
            j = order[t]
            f = min(r, int(b[j]))
            total += f * C[i, j]
            r -= f
        if iters < m:
            total += r * C[i, order[iters]]
        elif r:
            raise OracleError("ACT: target mass below source mass")
    return total


def act(X, mu_id, mu_m, nu_id, nu_m, Q: int, iters: int) -> float:
    """ACT-iters estimate of W1(mu, nu) (Section 4.1): the larger of the two
    one-way capacity-constrained relaxations, each source's mass moved as in
    ``_act_one_way``; Euclidean costs in float64, masses 2^-Q fixed point.
    iters = 0 is R-WMD (the paper states the two coincide)."""
    C = _dist_matrix(X, mu_id, nu_id)
    a = np.asarray(mu_m, np.int64)
    b = np.asarray(nu_m, np.int64)
    fwd = _act_one_way(C, a, b, iters)
    bwd = _act_one_way(C.T, b, a, iters)
    return max(fwd, bwd) / float(1 << Q)


def rwmd(X, mu_id, mu_m, nu_id, nu_m, Q: int) -> float:
    """Relaxed WMD (Section 1.1): every support point of one distribution
    sends its whole mass to its closest support point of the other; the
    larger of the two directions.  Written directly from that definition
    (row and column minima of the distance matrix), independent of ``act``."""
    C = _dist_matrix(X, mu_id, nu_id)
    a = np.asarray(mu_m, np.float64)
    b = np.asarray(nu_m, np.float64)
    return max(float(a @ C.min(axis=1)), float(b @ C.min(axis=0))) / float(1 << Q)


def act_pairs(X, q_off, q_id, q_m, d_off, d_id, d_m, pair_q, pair_d, Q: int, iters: int) -> np.ndarray:
    """``act`` for explicit (query, doc) pairs of CSR sets; float64 [n_pairs]."""
    out = np.empty(len(pair_q))
    for p, (q, d) in enumerate(zip(pair_q, pair_d)):
        qa, qb = q_off[q], q_off[q + 1]
        da, db = d_off[d], d_off[d + 1]
        out[p] = act(X, d_id[da:db], d_m[da:db], q_id[qa:qb], q_m[qa:qb], Q, iters)
    return out


# --------------------------------------------------------------------------
# Sinkhorn-k (Section 4.1 baseline; regularisation set per pair, appendix)
# --------------------------------------------------------------------------

def sinkhorn(X, mu_id, mu_m, nu_id, nu_m, Q: int, iters: int, eta: float = 30.0) -> float:
    """Sinkhorn-iters estimate of W1(mu, nu), float64.

    Reading: the Gibbs kernel is K = exp(-eta * C / M) with C the Euclidean
    cost matrix of the pair and M its largest entry (the appendix sets the
    regularisation from M with eta = 30 on every dataset).  Starting from
    v = 1, each iteration scales rows then columns, u = a / (K v) and
    v = b / (K^T u); the estimate is sum_ij u_i K_ij v_j C_ij.  A pair whose
    costs are all 0 (M = 0) has estimate 0."""
    C = _dist_matrix(X, mu_id, nu_id)
    a = np.asarray(mu_m, np.float64) / float(1 << Q)
    b = np.asarray(nu_m, np.float64) / float(1 << Q)
    M = C.max()
    if M == 0.0:
        return 0.0
    K = np.exp(-eta * C / M)
    v = np.ones(len(b))
    for _ in range(iters):
        u = a / (K @ v)
        v = b / (K.T @ u)
    return float(u @ ((K * C) @ v))


def sinkhorn_pairs(X, q_off, q_id, q_m, d_off, d_id, d_m, pair_q, pair_d, Q: int, iters: int,
                   eta: float = 30.0) -> np.ndarray:
    """``sinkhorn`` for explicit (query, doc) pairs of CSR sets; float64."""
    out = np.empty(len(pair_q))
    for p, (q, d) in enumerate(zip(pair_q, pair_d)):
        qa, qb = q_off[q], q_off[q + 1]
        da, db = d_off[d], d_off[d + 1]
        out[p] = sinkhorn(X, d_id[da:db], d_m[da:db], q_id[qa:qb], q_m[qa:qb], Q, iters, eta)
    return out
