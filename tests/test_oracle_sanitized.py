"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle.c is host code: it is built here with -fsanitize=address,undefined
(every UB check fatal), and a child Python process with the ASan runtime
preloaded drives every entry point of that build on small inputs -- the pin
battery of the mutation tests, the CSR batch helpers against the single-pair
calls they wrap, the eps-weighted Quadtree, exact W1 by successive shortest
paths, and the degenerate inputs (one point, every point coincident, a
distribution on one point).  A sanitizer report aborts the child; the test
checks its exit status and that its output holds no report.
"""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "oracle.c")

CHILD = textwrap.dedent("""
    import sys
    import numpy as np
    sys.path[:0] = [{root!r}, {tests!r}]
    import gen
    import oracle
    oracle._LIB = oracle.load({lib!r})
    from test_oracle_mutants import battery
    assert battery(oracle._LIB), "pin battery failed under the sanitizers"

    rng = np.random.default_rng(7)
    # CSR batch helpers against the single-pair calls, on a small world
    X = gen.gaussian_mixture(rng, 60, 4, 5, 0.3, False)
    t = oracle.Tree(X, gen.random_shift(rng, 4, 30), 30)
    Q = 16
    def dists(n, lo, hi):
        sizes = rng.integers(lo, hi + 1, n)
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        ids, ms = [], []
        for s in sizes:
            ids.append(rng.choice(60, s, replace=False))
            m = rng.integers(1, 100, s).astype(np.float64)
            m = np.floor(m / m.sum() * (1 << Q)).astype(np.int64)
            m[0] += (1 << Q) - m.sum()
            ms.append(m)
        return off, np.concatenate(ids).astype(np.uint32), np.concatenate(ms).astype(np.uint32)
    qo, qi, qm = dists(5, 1, 12)
    do, di, dm = dists(9, 1, 15)
    pq = np.repeat(np.arange(5), 9)
    pd = np.tile(np.arange(9), 5)
    U = t.quadtree_pairs(qo, qi, qm, do, di, dm, pq, pd, Q)
    F = t.flowtree_pairs(qo, qi, qm, do, di, dm, pq, pd, Q)
    for j, (a, b) in enumerate(zip(pq, pd)):
        args = (qi[qo[a]:qo[a + 1]], qm[qo[a]:qo[a + 1]], di[do[b]:do[b + 1]], dm[do[b]:do[b + 1]])
        assert U[j] == t.quadtree(*args, Q=Q)
        assert F[j] == t.flowtree(*args, Q=Q)[0]
        t.quadtree_eps(*args, Q=Q, eps=0.3)
        w = oracle.exact_w1_ssp(X, *args, Q=Q)
        assert w <= F[j] + 1e-9
    # one point; every point coincident; a distribution on one point
    one = oracle.Tree(np.zeros((1, 3), np.float32), np.ones(3, np.int64), 8)
    m1 = np.array([1 << Q], np.uint32)
    z = np.array([0], np.uint32)
    assert one.quadtree(z, m1, z, m1, Q=Q) == 0 and one.flowtree(z, m1, z, m1, Q=Q)[0] == 0.0
    Xc = np.ones((6, 2), np.float32)
    tc = oracle.Tree(Xc, np.ones(2, np.int64), 10)
    a = np.array([0, 3], np.uint32)
    b = np.array([5], np.uint32)
    ma = np.array([(1 << Q) - 5, 5], np.uint32)
    assert tc.quadtree(a, ma, b, m1, Q=Q) == 0 and tc.flowtree(a, ma, b, m1, Q=Q)[0] == 0.0
    print("sanitized oracle: all entry points clean")
""")


def _asan_runtime():
    if shutil.which("gcc") is None:
        pytest.skip("needs gcc")
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("the gcc here has no AddressSanitizer runtime")
    return asan


def _run_sanitized(tmp_path, text):
    """Build `text` (a copy of oracle.c) with the sanitizers and run the
    child driver on it; returns (exit status, stdout, all output)."""
    asan = _asan_runtime()
    src = str(tmp_path / "oracle.c")
    with open(src, "w") as f:
        f.write(text)
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-shared", "-fPIC", "-o", lib, src, "-lm"])
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "1"
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, tests=HERE, lib=lib)],
                       capture_output=True, text=True, env=env, timeout=600)
    return r.returncode, r.stdout, r.stdout + r.stderr


def test_oracle_clean_under_asan_ubsan(tmp_path):
    rc, stdout, out = _run_sanitized(tmp_path, open(SRC).read())
    assert rc == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "all entry points clean" in stdout


def test_sanitized_build_reports_a_planted_overflow(tmp_path):
    """The same run on a copy of oracle.c that writes one element past its
    duplicate-detection array for the largest point id: ASan must stop it
    (so the clean run above is a real check, not a build without the
    instrumentation)."""
    text = open(SRC).read()
    old = "t->pstamp[id[a]] = t->pstamp_id;"
    assert text.count(old) == 1
    rc, _, out = _run_sanitized(tmp_path, text.replace(old, "t->pstamp[id[a] + 1] = t->pstamp_id;"))
    assert rc != 0
    assert "AddressSanitizer: heap-buffer-overflow" in out, out[-4000:]
