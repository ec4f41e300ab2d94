"""Oracle Relaxed WMD and ACT-i against what the paper and the mathematics
fix, on tiny inputs.

Pins:
* hand-worked values (tests/golden/rwmd_act_hand.json, from the definitions
  of Section 1.1 and Section 4.1 and the one-dimensional W1 formula);
* ACT-0 == R-WMD (Section 4.1 says they coincide; the two oracle functions
  are written independently: row / column minima versus the sorted
  capacity walk);
* lower bounds: R-WMD <= ACT-1 <= ACT-2 <= ... <= W1 (Section 1.1: R-WMD is
  no larger than W1; each ACT iteration adds a constraint to a relaxation of
  the W1 program), W1 from the LP and from successive shortest paths;
* ACT with iterations >= support size - 1 equals the optimum of the
  relaxation that keeps the outflow of every source exact and caps every
  single edge by the target's mass, solved as an LP by HiGHS;
* single points: every estimate is ||x - y||; identical inputs give 0;
  symmetric in (mu, nu); exact scaling by 2 of the coordinates;
* a mutation battery: six plausible mistakes, each caught by a pin above.
"""
import json
import os

import numpy as np
import pytest

import gen
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "rwmd_act_hand.json")))
REAL_ONE_WAY = oracle._act_one_way


def random_pair(rng, V, s_mu, s_nu, Q):
    mu = rng.choice(V, size=s_mu, replace=False).astype(np.uint32)
    nu = rng.choice(V, size=s_nu, replace=False).astype(np.uint32)

    def masses(n):
        cuts = np.sort(rng.choice(np.arange(1, 1 << Q), size=n - 1, replace=False))
        return np.diff(np.concatenate([[0], cuts, [1 << Q]])).astype(np.uint32)
    return mu, masses(s_mu), nu, masses(s_nu)


def relaxed_lp(X, mu_id, mu_m, nu_id, nu_m, Q):
    """max over the two directions of: min sum f_ij C_ij subject to
    sum_j f_ij = a_i and 0 <= f_ij <= b_j (HiGHS)."""
    from scipy.optimize import linprog
    A = np.asarray(X, np.float64)
    C = np.sqrt(((A[np.asarray(mu_id, np.int64)][:, None, :] - A[np.asarray(nu_id, np.int64)][None, :, :]) ** 2).sum(-1))
    a = np.asarray(mu_m, np.float64) / 2.0 ** Q
    b = np.asarray(nu_m, np.float64) / 2.0 ** Q

    def one(C, a, b):
        n, m = C.shape
        Aeq = np.zeros((n, n * m))
        for i in range(n):
            Aeq[i, i * m:(i + 1) * m] = 1.0
        bounds = [(0.0, b[j]) for i in range(n) for j in range(m)]
        res = linprog(C.ravel(), A_eq=Aeq, b_eq=a, bounds=bounds, method="highs")
        assert res.status == 0
        return res.fun
    return max(one(C, a, b), one(C.T, b, a))


def world(seed, V=30, d=4):
    rng = np.random.default_rng(seed)
    return rng, gen.gaussian_mixture(rng, V, d, 3, 0.4, False)


@pytest.mark.parametrize("case", range(len(GOLD["cases"])))
def test_hand_values(case):
    c = GOLD["cases"][case]
    X = np.array(GOLD["X"], np.float32)
    Q = GOLD["Q"]
    args = (X, c["mu_id"], c["mu_m"], c["nu_id"], c["nu_m"], Q)
    assert oracle.rwmd(*args) == pytest.approx(c["rwmd"], abs=1e-12)
    assert oracle.act(*args, 0) == pytest.approx(c["rwmd"], abs=1e-12)
    assert oracle.act(*args, 1) == pytest.approx(c["act1"], abs=1e-12)
    if "act2" in c:
        assert oracle.act(*args, 2) == pytest.approx(c["act2"], abs=1e-12)
    assert oracle.exact_w1_lp(*args) == pytest.approx(c["w1"], abs=1e-9)


SIZES = [(1, 1), (1, 4), (3, 3), (5, 2), (6, 7), (8, 8)]


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("s_mu,s_nu", SIZES)
def test_chain_of_lower_bounds(seed, s_mu, s_nu):
    rng, X = world(seed)
    Q = 16
    mu_id, mu_m, nu_id, nu_m = random_pair(rng, len(X), s_mu, s_nu, Q)
    args = (X, mu_id, mu_m, nu_id, nu_m, Q)
    r = oracle.rwmd(*args)
    assert oracle.act(*args, 0) == pytest.approx(r, rel=1e-14, abs=1e-15)
    vals = [oracle.act(*args, i) for i in range(0, 9)]
    for lo, hi in zip(vals, vals[1:]):
        assert lo <= hi + 1e-12
    w1 = oracle.exact_w1_lp(*args)
    assert abs(oracle.exact_w1_ssp(*args) - w1) <= 1e-9 * max(1.0, w1)
    assert vals[-1] <= w1 + 1e-9
    # enough iterations: the full edge-capacity relaxation
    full = max(s_mu, s_nu) - 1
    assert oracle.act(*args, full) == pytest.approx(relaxed_lp(*args), rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_symmetry_identity_scaling(seed):
    rng, X = world(seed)
    Q = 16
    mu_id, mu_m, nu_id, nu_m = random_pair(rng, len(X), 5, 7, Q)
    for it in (0, 1, 3):
        v = oracle.act(X, mu_id, mu_m, nu_id, nu_m, Q, it)
        assert oracle.act(X, nu_id, nu_m, mu_id, mu_m, Q, it) == pytest.approx(v, rel=1e-14)
        assert oracle.act(2 * X, mu_id, mu_m, nu_id, nu_m, Q, it) == 2 * v
        assert oracle.act(X, mu_id, mu_m, mu_id, mu_m, Q, it) == 0.0
    assert oracle.rwmd(X, nu_id, nu_m, mu_id, mu_m, Q) == pytest.approx(oracle.rwmd(X, mu_id, mu_m, nu_id, nu_m, Q))


def test_single_points():
    rng, X = world(9)
    for x, y in [(0, 1), (3, 17), (5, 5)]:
        want = float(np.linalg.norm(X[x].astype(np.float64) - X[y]))
        one = [1 << 10]
        assert oracle.rwmd(X, [x], one, [y], one, 10) == pytest.approx(want, rel=1e-14, abs=0)
        for it in (0, 1, 5):
            assert oracle.act(X, [x], one, [y], one, 10, it) == pytest.approx(want, rel=1e-14, abs=0)


# -------------------------------------------------------------- mutants --

def _mut_no_capacity(C, a, b, iters):
    return sum(int(a[i]) * C[i].min() for i in range(C.shape[0]))


def _mut_rest_to_last_capped(C, a, b, iters):
    total = 0.0
    for i in range(C.shape[0]):
        order = np.argsort(C[i], kind="stable")
        r = int(a[i])
        for t in range(min(iters, C.shape[1])):
            f = min(r, int(b[order[t]]))
            total += f * C[i, order[t]]
            r -= f
        total += r * C[i, order[max(iters - 1, 0)]]
    return total


def _mut_capacity_from_source(C, a, b, iters):
    total = 0.0
    for i in range(C.shape[0]):
        order = np.argsort(C[i], kind="stable")
        r = int(a[i])
        for t in range(min(iters, C.shape[1])):
            f = min(r, int(a[i]) // 2)
            total += f * C[i, order[t]]
            r -= f
        if iters < C.shape[1]:
            total += r * C[i, order[iters]]
    return total


def _mut_farthest_first(C, a, b, iters):
    return REAL_ONE_WAY(-C, a, b, iters) * -1.0


def _mut_rwmd_smaller_side(X, mu_id, mu_m, nu_id, nu_m, Q):
    A = np.asarray(X, np.float64)
    C = np.sqrt(((A[np.asarray(mu_id, np.int64)][:, None, :] - A[np.asarray(nu_id, np.int64)][None, :, :]) ** 2).sum(-1))
    a, b = np.asarray(mu_m, np.float64), np.asarray(nu_m, np.float64)
    return min(a @ C.min(1), b @ C.min(0)) / 2.0 ** Q


MUTANTS = {
    "R-WMD takes the smaller direction": ("rwmd", _mut_rwmd_smaller_side),
    "no capacity": ("_act_one_way", _mut_no_capacity),
    "rest to the last capped target": ("_act_one_way", _mut_rest_to_last_capped),
    "capacity from the source": ("_act_one_way", _mut_capacity_from_source),
    "farthest first": ("_act_one_way", _mut_farthest_first),
}


def pins_pass():
    try:
        for case in range(len(GOLD["cases"])):
            test_hand_values(case)
        for seed in range(3):
            for s_mu, s_nu in SIZES:
                test_chain_of_lower_bounds(seed, s_mu, s_nu)
    except (AssertionError, oracle.OracleError, ValueError, IndexError):
        return False
    return True


@pytest.mark.parametrize("name", sorted(MUTANTS) + ["one direction only"])
def test_mutants_are_caught(name, monkeypatch):
    if name == "one direction only":
        real = REAL_ONE_WAY
        calls = {"n": 0}

        def fwd_only(C, a, b, iters):
            calls["n"] += 1
            return real(C, a, b, iters) if calls["n"] % 2 == 1 else 0.0
        monkeypatch.setattr(oracle, "_act_one_way", fwd_only)
    else:
        attr, fn = MUTANTS[name]
        monkeypatch.setattr(oracle, attr, fn)
    assert not pins_pass(), "mutant '%s' passed every pin" % name


def test_unmutated_pins_pass():
    assert pins_pass()
