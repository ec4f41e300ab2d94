"""Seeded synthetic inputs shared by the CPU oracle tests and the GPU path.

This module only draws inputs: ground points, supports, fixed-point masses and
the random shift of the quadtree.  It holds none of the estimators'
arithmetic.  Everything is drawn from ``numpy.random.default_rng(seed)``
(PCG64) so the same seed gives the same bytes on every machine.

Shapes follow the paper's workloads (Section 4, dataset table): word-embedding
ground sets with documents that are uniform over their distinct words, and the
28x28 pixel grid with greyscale images.  The real datasets are not used; the
stand-ins below reproduce their shape (support sizes, dimension, clustering).

Fixed-point masses: every distribution's masses are positive integers that sum
to exactly 2**Q.  A uniform distribution over m ids gets floor(2**Q / m) per id
and the first (2**Q mod m) ids in ascending id order get one more unit.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass, field

import numpy as np

B_DEFAULT = 30

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None
_LIB_LOCK = threading.Lock()


def build_sampler(force: bool = False) -> str:
    """Compile the sampling helper with gcc into this folder; return its path."""
    src = os.path.join(_HERE, "_sample.c")
    out = os.path.join(_HERE, "_libgen.so")
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, src])
        os.replace(tmp, out)
    return out


def _lib():
    global _LIB
    with _LIB_LOCK:
        if _LIB is None:
            lib = ctypes.CDLL(build_sampler())
            p = ctypes.c_void_p
            i64 = ctypes.c_int64
            lib.gen_build_guide.argtypes = [p, i64, i64, p]
            lib.gen_build_guide.restype = None
            lib.gen_first_distinct.argtypes = [p, i64, p, i64, p, i64, p, p, p, i64, i64, p, p]
            lib.gen_first_distinct.restype = i64
            lib.gen_uniform_masses.argtypes = [p, p, i64, ctypes.c_int32, p, p]
            lib.gen_uniform_masses.restype = i64
            _LIB = lib
    return _LIB


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


# --------------------------------------------------------------------------
# Ground sets
# --------------------------------------------------------------------------

def gaussian_mixture(rng, V: int, d: int, n_clusters: int, sigma: float,
                     normalize: bool) -> np.ndarray:
    """V points in R^d: centre ~ N(0, I), cluster uniform, x = c + sigma*N(0, I).

    With ``normalize`` every row is scaled to unit L2 norm (in float64) before
    the cast to float32, like word embeddings compared by direction.
    """
    centers = rng.standard_normal((n_clusters, d))
    labels = rng.integers(0, n_clusters, size=V)
    X = np.empty((V, d), dtype=np.float32)
    step = 16384
    for a in range(0, V, step):
        b = min(V, a + step)
        x = centers[labels[a:b]] + sigma * rng.standard_normal((b - a, d))
        if normalize:
            x /= np.linalg.norm(x, axis=1, keepdims=True)
        X[a:b] = x.astype(np.float32)
    return X


def pixel_grid(side: int = 28) -> np.ndarray:
    """The points (i, j), i, j = 1..side, as float32; id = (i-1)*side + (j-1)."""
    i, j = np.meshgrid(np.arange(1, side + 1), np.arange(1, side + 1), indexing="ij")
    return np.stack([i.ravel(), j.ravel()], axis=1).astype(np.float32)


def random_shift(rng, d: int, B: int = B_DEFAULT) -> np.ndarray:
    """Integer shift s_i uniform in [1, 2**(B-1)] per dimension (int64).

    In grid units of 2*Phi / 2**B this is the paper's shift sigma_i in (0, Phi]
    (Section 2); the open lower end keeps every grid code inside [0, 2**B).
    """
    return rng.integers(1, (1 << (B - 1)) + 1, size=d, dtype=np.int64)


# --------------------------------------------------------------------------
# Supports and masses
# --------------------------------------------------------------------------

def zipf_cdf(V: int, a: float = 1.1) -> np.ndarray:
    w = np.arange(1, V + 1, dtype=np.float64) ** (-a)
    c = np.cumsum(w)
    return c / c[-1]


def zipf_distinct(rng, sizes: np.ndarray, V: int, a: float = 1.1):
    """Supports of ``sizes[j]`` distinct ids each, drawn Zipf(a) over ids 0..V-1.

    Id i has draw probability proportional to (i+1)**-a; each support is the
    first sizes[j] distinct ids of an i.i.d. draw sequence, documents taking
    consecutive stretches of one uniform stream.  Returns (off int64[n+1],
    ids uint32[nnz]) with ids in first-appearance order.
    """
    sizes = np.asarray(sizes, dtype=np.int64)
    if np.any(sizes > V) or np.any(sizes < 0):
        raise ValueError("support sizes must lie in [0, V]")
    n = len(sizes)
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    ids = np.empty(int(off[-1]), dtype=np.uint32)
    cdf = zipf_cdf(V, a)
    G = max(1024, V)
    guide = np.empty(G, dtype=np.int64)
    lib = _lib()
    lib.gen_build_guide(_ptr(cdf), V, G, _ptr(guide))
    stamp = np.zeros(V, dtype=np.int64)
    pos = ctypes.c_int64(0)
    u = np.empty(0, dtype=np.float64)
    doc = 0
    while doc < n:
        # roughly 2.2 draws per distinct id at these sizes; top up as needed
        want = int(2.4 * int(off[-1] - off[doc])) + 4096
        u = np.concatenate([u[pos.value:], rng.random(want)])
        pos = ctypes.c_int64(0)
        doc = lib.gen_first_distinct(_ptr(cdf), V, _ptr(guide), G, _ptr(u), len(u),
                                     ctypes.byref(pos), _ptr(sizes), _ptr(off), doc, n,
                                     _ptr(ids), _ptr(stamp))
    return off, ids


def uniform_masses(off: np.ndarray, ids: np.ndarray, Q: int) -> np.ndarray:
    """Uniform fixed-point masses summing to 2**Q per distribution.

    floor(2**Q / m) each; the first (2**Q mod m) ids in ascending id order get
    one extra unit.
    """
    off = np.ascontiguousarray(off, dtype=np.int64)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    n = len(off) - 1
    mass = np.empty(len(ids), dtype=np.uint32)
    smax = int(np.diff(off).max()) if n else 0
    scratch = np.empty(max(1, smax), dtype=np.uint32)
    if _lib().gen_uniform_masses(_ptr(off), _ptr(ids), n, Q, _ptr(mass), _ptr(scratch)) != 0:
        raise ValueError("empty support")
    return mass


def sizes_uniform(rng, n: int, lo: int, hi: int) -> np.ndarray:
    return rng.integers(lo, hi + 1, size=n).astype(np.int64)


def sizes_power(rng, n: int, lo: int, hi: int, a: float = 1.1) -> np.ndarray:
    """Support sizes m in {lo..hi} with P(m) proportional to m**-a."""
    m = np.arange(lo, hi + 1, dtype=np.float64)
    c = np.cumsum(m ** (-a))
    c /= c[-1]
    return (lo + np.searchsorted(c, rng.random(n), side="right")).astype(np.int64)


def _segment_dist2(px, py, ax, ay, bx, by):
    """Squared distance from pixel centres to segments (broadcast)."""
    vx, vy = bx - ax, by - ay
    wx, wy = px - ax, py - ay
    L2 = vx * vx + vy * vy
    t = np.where(L2 > 0, (wx * vx + wy * vy) / np.where(L2 > 0, L2, 1.0), 0.0)
    t = np.clip(t, 0.0, 1.0)
    dx = wx - t * vx
    dy = wy - t * vy
    return dx * dx + dy * dy


def stroke_images(rng, n: int, side: int = 28, Q: int = 16, n_lo: int = 100,
                  n_hi: int = 200, blur: float = 1.0):
    """Greyscale images over the side x side pixel grid, as fixed-point masses.

    Each image: 1-3 line strokes between endpoints uniform in [1, side]^2,
    intensity sum_s exp(-dist(p, stroke_s)^2 / (2 blur^2)); the n ~ U{n_lo..n_hi}
    brightest pixels are kept (ties to the lower pixel id), normalised, and
    rounded to 2**Q units by largest remainder (ties to the lower pixel id);
    a pixel rounded to 0 gets one unit taken from the largest mass.
    Returns (off, ids, mass) with ids ascending inside each image.
    """
    P = side * side
    grid = pixel_grid(side).astype(np.float64)
    px, py = grid[:, 0][None, :], grid[:, 1][None, :]
    n_str = rng.integers(1, 4, size=n)
    ends = rng.uniform(1.0, float(side), size=(n, 3, 4))
    keep = rng.integers(n_lo, n_hi + 1, size=n)
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(keep, out=off[1:])
    ids = np.empty(int(off[-1]), dtype=np.uint32)
    mass = np.empty(int(off[-1]), dtype=np.uint32)
    total = 1 << Q
    step = 4096
    pid = np.arange(P)
    for a in range(0, n, step):
        b = min(n, a + step)
        inten = np.zeros((b - a, P))
        for s in range(3):
            e = ends[a:b, s]
            d2 = _segment_dist2(px, py, e[:, 0:1], e[:, 1:2], e[:, 2:3], e[:, 3:4])
            inten += np.where((n_str[a:b] > s)[:, None], np.exp(-d2 / (2.0 * blur * blur)), 0.0)
        for r in range(b - a):
            j = a + r
            m = int(keep[j])
            order = np.lexsort((pid, -inten[r]))[:m]
            sel = np.sort(order)
            w = inten[r, sel]
            w = w / w.sum()
            x = w * total
            base = np.floor(x).astype(np.int64)
            rem = total - int(base.sum())
            frac = x - base
            if rem > 0:
                give = np.lexsort((sel, -frac))[:rem]
                base[give] += 1
            while True:
                z = np.flatnonzero(base == 0)
                if len(z) == 0:
                    break
                big = int(np.lexsort((sel, -base))[0])
                base[big] -= 1
                base[z[0]] += 1
            assert base.sum() == total and base.min() >= 1
            ids[off[j]:off[j + 1]] = sel
            mass[off[j]:off[j + 1]] = base
    return off, ids, mass


# --------------------------------------------------------------------------
# The paper's random model (Section 3.2)
# --------------------------------------------------------------------------

def _unit_rows(x):
    return x / np.linalg.norm(x, axis=-1, keepdims=True)


def sphere_cap_point(rng, x: np.ndarray, eps: float) -> np.ndarray:
    """A point uniform on the unit sphere among those within distance eps of x.

    The polar angle t to x has density proportional to sin(t)**(d-2) on
    [0, tmax], tmax = 2 asin(eps / 2); it is drawn by rejection from the
    uniform law on [0, tmax], then a uniform direction orthogonal to x.
    """
    d = len(x)
    tmax = 2.0 * np.arcsin(min(1.0, eps / 2.0))
    while True:
        t = rng.uniform(0.0, tmax)
        if d == 2 or rng.random() <= (np.sin(t) / np.sin(tmax)) ** (d - 2):
            break
    v = rng.standard_normal(d)
    v -= v.dot(x) * x
    v = v / np.linalg.norm(v)
    return np.cos(t) * x + np.sin(t) * v


def random_model(rng, N: int, d: int, s: int, eps: float):
    """Ground set of N uniform points on S^{d-1}, one planted doc and its query.

    Returns (X float32 [(N+s), d], doc_ids, query_ids): the planted doc is
    uniform over s of the first N points, the query is uniform over the s
    extra points y_k, each uniform in the eps-cap around its x_k.
    """
    X = _unit_rows(rng.standard_normal((N, d)))
    planted = rng.choice(N, size=s, replace=False)
    Y = np.stack([sphere_cap_point(rng, X[k], eps) for k in planted])
    G = np.vstack([X, Y]).astype(np.float32)
    return G, planted.astype(np.uint32), np.arange(N, N + s, dtype=np.uint32)


def random_model_swaps(rng, N: int, d: int, s: int, eps: float, Q: int = 24, B: int = None):
    """One repetition of the random model of Section 3.2, with the planted
    doc's single-swap neighbours as its competitors.

    Ground set: the N sphere points and the s query points y_k.  Doc 0 is the
    planted doc (support x_1..x_s); docs 1.. replace one x_k by another of the
    N points, for every k and every such point: s * (N - s) docs.  Masses
    follow the support position, floor(2^Q / s) each and one more unit for
    the first (2^Q mod s) positions, so a swapped point carries exactly the
    mass of the point it replaces and y_k that of x_k.
    """
    B = B_DEFAULT if B is None else B
    G, planted, qids = random_model(rng, N, d, s, eps)
    m = np.full(s, (1 << Q) // s, np.uint32)
    m[: (1 << Q) % s] += 1
    others = np.setdiff1d(np.arange(N, dtype=np.uint32), planted)
    n_docs = 1 + s * len(others)
    ids = np.empty((n_docs, s), np.uint32)
    ids[0] = planted
    for k in range(s):
        blk = ids[1 + k * len(others): 1 + (k + 1) * len(others)]
        blk[:] = planted
        blk[:, k] = others
    doc_off = np.arange(n_docs + 1, dtype=np.int64) * s
    ds = Dataset("random_model", G, random_shift(rng, d, B), B, Q, doc_off, ids.reshape(-1),
                 np.tile(m, n_docs), np.array([0, s], np.int64), qids, m.copy(), 2)
    ds.extra["planted"] = planted
    return ds


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

@dataclass
class Dataset:
    name: str
    X: np.ndarray            # float32 [V, d]
    shift: np.ndarray        # int64 [d], in [1, 2**(B-1)]
    B: int
    Q: int
    doc_off: np.ndarray      # int64 [n_docs + 1]
    doc_id: np.ndarray       # uint32 [nnz]
    doc_mass: np.ndarray     # uint32 [nnz]
    q_off: np.ndarray
    q_id: np.ndarray
    q_mass: np.ndarray
    k: int = 10
    extra: dict = field(default_factory=dict)

    @property
    def V(self):
        return self.X.shape[0]

    @property
    def d(self):
        return self.X.shape[1]

    @property
    def n_docs(self):
        return len(self.doc_off) - 1

    @property
    def n_queries(self):
        return len(self.q_off) - 1


def _text_like(name, rng, V, d, n_clusters, sigma, normalize, size_fn, n_docs,
               n_queries, Q, B, k, extra=None):
    X = gaussian_mixture(rng, V, d, n_clusters, sigma, normalize)
    dsz = size_fn(rng, n_docs)
    doff, dids = zipf_distinct(rng, dsz, V)
    qsz = size_fn(rng, n_queries)
    qoff, qids = zipf_distinct(rng, qsz, V)
    shift = random_shift(rng, d, B)
    return Dataset(name, X, shift, B, Q, doff, dids, uniform_masses(doff, dids, Q),
                   qoff, qids, uniform_masses(qoff, qids, Q), k, extra or {})


def make(name: str, seed: int = 0, **over) -> Dataset:
    """Build a named workload.  Keyword overrides shrink it for tests.

    tiny   : V=2000, R^16, 20-cluster mixture (sigma 0.1); 500 docs and 10
             queries uniform over 10..30 distinct Zipf(1.1) points; top-5.
    text   : V=100k, R^300, L2-normalised 200-cluster mixture (sigma 0.1);
             100k docs and 1000 queries over 20..200 distinct words; prune to
             1000 by Quadtree, rerank to 20 by Flowtree.
    image  : 28x28 grid in R^2; 60k stroke images and 1000 queries with
             100..200 pixels, masses in units of 2**-16; top-10.
    batched: the text ground space with 1M docs and 4096 queries whose sizes
             follow P(m) ~ m**-1.1 on 5..500; prune to 1000, rerank to 20.
    grad   : V=50k in R^300 (text law); 256 (query, doc) pairs with sizes
             20..200.
    """
    rng = np.random.default_rng(seed)
    B = over.pop("B", B_DEFAULT)
    if name == "tiny":
        p = dict(V=2000, d=16, n_docs=500, n_queries=10, lo=10, hi=30, Q=24, k=5)
        p.update(over)
        return _text_like(name, rng, p["V"], p["d"], 20, 0.1, False,
                          lambda r, n: sizes_uniform(r, n, p["lo"], p["hi"]),
                          p["n_docs"], p["n_queries"], p["Q"], B, p["k"])
    if name == "text":
        p = dict(V=100_000, d=300, n_docs=100_000, n_queries=1000, lo=20, hi=200, Q=24,
                 k=20, prune=1000)
        p.update(over)
        return _text_like(name, rng, p["V"], p["d"], 200, 0.1, True,
                          lambda r, n: sizes_uniform(r, n, p["lo"], p["hi"]),
                          p["n_docs"], p["n_queries"], p["Q"], B, p["k"],
                          {"prune": p["prune"]})
    if name == "batched":
        p = dict(V=100_000, d=300, n_docs=1_000_000, n_queries=4096, lo=5, hi=500, Q=24,
                 k=20, prune=1000)
        p.update(over)
        return _text_like(name, rng, p["V"], p["d"], 200, 0.1, True,
                          lambda r, n: sizes_power(r, n, p["lo"], p["hi"]),
                          p["n_docs"], p["n_queries"], p["Q"], B, p["k"],
                          {"prune": p["prune"]})
    if name == "image":
        p = dict(n_docs=60_000, n_queries=1000, Q=16, k=10, lo=100, hi=200)
        p.update(over)
        X = pixel_grid(28)
        doff, dids, dm = stroke_images(rng, p["n_docs"], Q=p["Q"], n_lo=p["lo"], n_hi=p["hi"])
        qoff, qids, qm = stroke_images(rng, p["n_queries"], Q=p["Q"], n_lo=p["lo"], n_hi=p["hi"])
        shift = random_shift(rng, 2, B)
        return Dataset(name, X, shift, B, p["Q"], doff, dids, dm, qoff, qids, qm, p["k"])
    if name == "grad":
        p = dict(V=50_000, d=300, n_pairs=256, lo=20, hi=200, Q=24)
        p.update(over)
        ds = _text_like(name, rng, p["V"], p["d"], 200, 0.1, True,
                        lambda r, n: sizes_uniform(r, n, p["lo"], p["hi"]),
                        p["n_pairs"], p["n_pairs"], p["Q"], B, 1)
        ds.extra["pair_q"] = np.arange(p["n_pairs"], dtype=np.int64)
        ds.extra["pair_d"] = np.arange(p["n_pairs"], dtype=np.int64)
        return ds
    raise KeyError(name)
