"""Oracle Sinkhorn-k against what the paper and the mathematics fix, on tiny
inputs.

Pins:
* hand-worked values (tests/golden/sinkhorn_hand.json) for one and two
  iterations;
* a side with one support point: one iteration already gives the exact W1
  (every coupling of a point mass is the product coupling), for any eta;
* eta -> 0: the kernel is all ones and one iteration returns the product
  coupling's cost a^T C b;
* converged iterations sit within the entropic bias of W1:
  W1 - 1e-9 <= S <= W1 + M ln(n m) / eta (the kernel is exp(-eta C / M), so
  the regularisation is M / eta), W1 from the LP;
* scaling the coordinates by 2 doubles the estimate exactly (the kernel
  depends on C / M only);
* four mutants, each caught.
"""
import json
import os

import numpy as np
import pytest

import gen
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "sinkhorn_hand.json")))
REAL = oracle.sinkhorn


def random_pair(rng, V, s_mu, s_nu, Q):
    mu = rng.choice(V, size=s_mu, replace=False).astype(np.uint32)
    nu = rng.choice(V, size=s_nu, replace=False).astype(np.uint32)

    def masses(n):
        cuts = np.sort(rng.choice(np.arange(1, 1 << Q), size=n - 1, replace=False))
        return np.diff(np.concatenate([[0], cuts, [1 << Q]])).astype(np.uint32)
    return mu, masses(s_mu), nu, masses(s_nu)


def world(seed, V=30, d=4):
    rng = np.random.default_rng(seed)
    return rng, gen.gaussian_mixture(rng, V, d, 3, 0.4, False)


def cost_matrix(X, a_id, b_id):
    A = np.asarray(X, np.float64)
    return np.sqrt(((A[np.asarray(a_id, np.int64)][:, None, :] - A[np.asarray(b_id, np.int64)][None, :, :]) ** 2).sum(-1))


@pytest.mark.parametrize("case", range(len(GOLD["cases"])))
def test_hand_values(case):
    c = GOLD["cases"][case]
    X = np.array(GOLD["X"], np.float32)
    v = oracle.sinkhorn(X, GOLD["mu_id"], GOLD["mu_m"], GOLD["nu_id"], GOLD["nu_m"], GOLD["Q"], c["iters"], GOLD["eta"])
    assert v == pytest.approx(c["value"], rel=1e-12)


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("iters", [1, 3])
def test_point_mass_side_is_exact(seed, iters):
    rng, X = world(seed)
    Q = 16
    mu_id, mu_m, nu_id, nu_m = random_pair(rng, len(X), 1, 6, Q)
    want = float(cost_matrix(X, mu_id, nu_id)[0] @ (nu_m / 2.0 ** Q))
    for eta in (30.0, 3.0):
        assert oracle.sinkhorn(X, mu_id, mu_m, nu_id, nu_m, Q, iters, eta) == pytest.approx(want, rel=1e-12)
        assert oracle.sinkhorn(X, nu_id, nu_m, mu_id, mu_m, Q, iters, eta) == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("seed", range(5))
def test_vanishing_eta_is_product_coupling(seed):
    rng, X = world(seed)
    Q = 16
    mu_id, mu_m, nu_id, nu_m = random_pair(rng, len(X), 5, 7, Q)
    want = float((mu_m / 2.0 ** Q) @ cost_matrix(X, mu_id, nu_id) @ (nu_m / 2.0 ** Q))
    assert oracle.sinkhorn(X, mu_id, mu_m, nu_id, nu_m, Q, 1, 1e-9) == pytest.approx(want, rel=1e-8)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("s_mu,s_nu", [(3, 3), (4, 6), (7, 5)])
def test_converged_within_entropic_bias(seed, s_mu, s_nu):
    rng, X = world(seed)
    Q = 16
    mu_id, mu_m, nu_id, nu_m = random_pair(rng, len(X), s_mu, s_nu, Q)
    args = (X, mu_id, mu_m, nu_id, nu_m, Q)
    w1 = oracle.exact_w1_lp(*args)
    M = cost_matrix(X, mu_id, nu_id).max()
    s = oracle.sinkhorn(*args, 3000, 30.0)
    assert w1 - 1e-9 <= s <= w1 + M * np.log(s_mu * s_nu) / 30.0


@pytest.mark.parametrize("seed", range(3))
def test_scaling(seed):
    rng, X = world(seed)
    Q = 16
    mu_id, mu_m, nu_id, nu_m = random_pair(rng, len(X), 5, 4, Q)
    for iters in (1, 3):
        v = oracle.sinkhorn(X, mu_id, mu_m, nu_id, nu_m, Q, iters)
        assert oracle.sinkhorn(2 * X, mu_id, mu_m, nu_id, nu_m, Q, iters) == pytest.approx(2 * v, rel=1e-14)


# -------------------------------------------------------------- mutants --

def _kernel_without_M(X, mu_id, mu_m, nu_id, nu_m, Q, iters, eta=30.0):
    C = cost_matrix(X, mu_id, nu_id)
    a, b = np.asarray(mu_m) / 2.0 ** Q, np.asarray(nu_m) / 2.0 ** Q
    K = np.exp(-eta * C)
    v = np.ones(len(b))
    for _ in range(iters):
        u = a / (K @ v)
        v = b / (K.T @ u)
    return float(u @ ((K * C) @ v))


def _columns_first(X, mu_id, mu_m, nu_id, nu_m, Q, iters, eta=30.0):
    C = cost_matrix(X, mu_id, nu_id)
    a, b = np.asarray(mu_m) / 2.0 ** Q, np.asarray(nu_m) / 2.0 ** Q
    M = C.max()
    K = np.exp(-eta * C / M)
    u = np.ones(len(a))
    for _ in range(iters):
        v = b / (K.T @ u)
        u = a / (K @ v)
    return float(u @ ((K * C) @ v))


def _mass_not_cost(X, mu_id, mu_m, nu_id, nu_m, Q, iters, eta=30.0):
    C = cost_matrix(X, mu_id, nu_id)
    a, b = np.asarray(mu_m) / 2.0 ** Q, np.asarray(nu_m) / 2.0 ** Q
    K = np.exp(-eta * C / C.max())
    v = np.ones(len(b))
    for _ in range(iters):
        u = a / (K @ v)
        v = b / (K.T @ u)
    return float(u @ K @ v)


def _one_iteration_short(X, mu_id, mu_m, nu_id, nu_m, Q, iters, eta=30.0):
    return REAL(X, mu_id, mu_m, nu_id, nu_m, Q, max(iters - 1, 0) or 1, eta) if iters > 1 else \
        REAL(X, mu_id, mu_m, nu_id, nu_m, Q, 2, eta)


MUTANTS = {"kernel without M": _kernel_without_M, "columns first": _columns_first,
           "mass instead of cost": _mass_not_cost, "iteration count off by one": _one_iteration_short}


def pins_pass():
    try:
        for case in range(len(GOLD["cases"])):
            test_hand_values(case)
        for seed in range(2):
            test_point_mass_side_is_exact(seed, 1)
            test_scaling(seed)
            test_converged_within_entropic_bias(seed, 4, 6)
    except (AssertionError, ValueError, FloatingPointError):
        return False
    return True


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutants_are_caught(name, monkeypatch):
    monkeypatch.setattr(oracle, "sinkhorn", MUTANTS[name])
    assert not pins_pass(), "mutant '%s' passed every pin" % name


def test_unmutated_pins_pass():
    assert pins_pass()
