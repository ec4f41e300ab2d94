"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of oracle.c (a dropped term, a wrong
sign, index or order, a transposed operand), builds it on the CPU and runs a
compact battery of the pins used by the other oracle tests.  The battery
passes on the real oracle and must fail on every mutant.
"""
import json
import os
import subprocess

import numpy as np
import pytest

import gen
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "oracle.c")

MUTANTS = {
    "edge weight one level too heavy": (
        "s += (unsigned __int128)a << (t->B - t->depth[v]);",
        "s += (unsigned __int128)a << (t->B - t->depth[v] + 1);"),
    "query mass added instead of subtracted": (
        "t->acc[v] += side ? -(int64_t)m[a] : (int64_t)m[a];",
        "t->acc[v] += (int64_t)m[a];"),
    "dimensions compared last-first": (
        "out[i / 64] |= bit << (63 - (i % 64));",
        "{ int j = t->d - 1 - i; out[j / 64] |= bit << (63 - (j % 64)); }"),
    "leaves pass up without matching": (
        "while (i < cm && j < cn) {",
        "while (i < cm && j < cn && t->first_rank[v] != t->last_rank[v]) {"),
    # (reversing BOTH lists is not a mistake: the front-to-front matching of
    # two lists equals that of the two reversed lists)
    "query items matched in descending Morton rank": (
        "qsort(ln, cn, sizeof(item_t*), cmp_rank);",
        "qsort(ln, cn, sizeof(item_t*), cmp_rank);"
        " for (int64_t r = 0; r < cn / 2; ++r) {"
        " item_t* x = ln[r]; ln[r] = ln[cn - 1 - r]; ln[cn - 1 - r] = x; }"),
    "distance squared instead of the norm": (
        "s += (double)em_eta[e] * sqrt(acc);",
        "s += (double)em_eta[e] * acc;"),
    "cost always against the first query point": (
        "const float* y = X + (int64_t)nu_id[em_nu[e]] * t->d;",
        "const float* y = X + (int64_t)nu_id[0] * t->d;"),
    "grid twice too coarse": (
        "t->scale = phi > 0.0 ? half / phi : 0.0;",
        "t->scale = phi > 0.0 ? half / (2.0 * phi) : 0.0;"),
    "two-point cells made leaves": (
        "if (n == 1 || k == t->B) {",
        "if (n <= 2 || k == t->B) {"),
    "both pointers always advance": (
        "if (lm[i]->resid == 0) ++i;\n      if (ln[j]->resid == 0) ++j;",
        "++i;\n      ++j;"),
}


def build_variant(tmp_path, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, "mutation anchor must appear exactly once: %r" % old
    src = os.path.join(tmp_path, "oracle.c")
    with open(src, "w") as f:
        f.write(text.replace(old, new))
    out = os.path.join(tmp_path, "liboracle_variant.so")
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-shared", "-fPIC", "-o", out, src, "-lm"])
    return oracle.load(out)


def battery(lib):
    """True when every pin holds for the library."""
    try:
        # hand-worked fixtures
        for name in ("hand_1d.json", "hand_2d_order.json"):
            g = json.load(open(os.path.join(HERE, "golden", name)))
            X = np.array(g["X"], np.float32)
            t = oracle.Tree(X, np.array(g["shift"]), g["B"], lib=lib)
            ex = t.export()
            if ex["code"].tolist() != g["codes"] or ex["rank_of"].tolist() != g["rank_of"]:
                return False
            for c in g["cases"]:
                args = (c["mu_id"], c["mu_m"], c["nu_id"], c["nu_m"])
                if t.quadtree(*args, Q=g["Q"]) != c["quadtree_units"]:
                    return False
                cost, _ = t.flowtree(*args, Q=g["Q"])
                if abs(cost - c["flowtree"]) > 1e-12:
                    return False
        # random tiny worlds: tree-LP, flow properties, W1 bound, bracket
        for seed in range(4):
            rng = np.random.default_rng(seed)
            X = gen.gaussian_mixture(rng, 40, 3, 4, 0.3, False)
            t = oracle.Tree(X, gen.random_shift(rng, 3, 30), 30, lib=lib)
            Q = 12
            for (sm, sn, shared) in ((3, 5, 0), (6, 6, 3)):
                mu = rng.choice(40, sm, replace=False).astype(np.uint32)
                nu = rng.choice(40, sn, replace=False).astype(np.uint32)
                nu[:shared] = mu[:shared]
                mm = np.full(sm, (1 << Q) // sm, np.uint32); mm[0] += (1 << Q) - mm.sum()
                nm = np.full(sn, (1 << Q) // sn, np.uint32); nm[0] += (1 << Q) - nm.sum()
                U = t.quadtree(mu, mm, nu, nm, Q=Q)
                if U != round(oracle.tree_w1_lp(t, mu, mm, nu, nm, Q) * (1 << Q)):
                    return False
                cost, fl = t.flowtree(mu, mm, nu, nm, Q=Q)
                if np.bincount(fl["mu"], weights=fl["eta"], minlength=sm).tolist() != mm.tolist():
                    return False
                if np.bincount(fl["nu"], weights=fl["eta"], minlength=sn).tolist() != nm.tolist():
                    return False
                tc = sum(int(e) * t.tree_dist(mu[a], nu[b]) for a, b, e in zip(fl["mu"], fl["nu"], fl["eta"]))
                if tc != U:
                    return False
                if cost < oracle.exact_w1_lp(X, mu, mm, nu, nm, Q=Q) - 1e-9:
                    return False
                lo, hi = oracle.flow_face_bracket(t, mu, mm, nu, nm, Q)
                if not (lo - 1e-7 <= cost <= hi + 1e-7):
                    return False
        return True
    except oracle.OracleError:
        return False


def test_battery_passes_on_oracle():
    assert battery(oracle._lib())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_battery_catches_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    lib = build_variant(str(tmp_path), old, new)
    assert not battery(lib), "pins did not catch: " + name
