"""Oracle gradient of the Flowtree cost with the tree and flow pattern frozen.

The paper defines no gradient; the reading (documented in
oracle.frozen_cost) makes the cost a function C(X, mu_w, nu_w) that is
smooth in X away from coincident points and linear in the weights.  Pins:
* central finite differences (h = 1e-3, float64) of C in X;
* finite differences of C in the weights (exact up to rounding: C is linear);
* a single point pair: the gradient is (x - y) / ||x - y||;
* moving one mass unit between two items of one side through the real
  (unfrozen) greedy changes the cost by the difference of their adjoints,
  whenever the greedy's pattern does not change.
"""
import numpy as np
import pytest

import gen
import oracle


def world(seed, V=60, d=5):
    rng = np.random.default_rng(seed)
    X = gen.gaussian_mixture(rng, V, d, 4, 0.3, False)
    t = oracle.Tree(X, gen.random_shift(rng, d, 30), 30)
    return rng, X, t


def pair(rng, V, s_mu, s_nu, Q):
    mu = rng.choice(V, s_mu, replace=False).astype(np.uint32)
    nu = rng.choice(V, s_nu, replace=False).astype(np.uint32)
    def masses(n):
        cuts = np.sort(rng.choice(np.arange(1, 1 << Q), size=n - 1, replace=False))
        return np.diff(np.concatenate([[0], cuts, [1 << Q]])).astype(np.uint32)
    return mu, masses(s_mu), nu, masses(s_nu)


@pytest.mark.parametrize("seed", range(6))
def test_frozen_cost_equals_flowtree(seed):
    rng, X, t = world(seed)
    Q = 16
    mu, mm, nu, nm = pair(rng, len(X), 7, 5, Q)
    c, fl = t.flowtree(mu, mm, nu, nm, Q=Q)
    cf = oracle.frozen_cost(X, mu, nu, fl, mm / 2.0 ** Q, nm / 2.0 ** Q)
    assert cf == pytest.approx(c, rel=1e-13)


@pytest.mark.parametrize("seed", range(6))
def test_grad_coordinates_fd(seed):
    rng, X, t = world(seed)
    Q = 16
    mu, mm, nu, nm = pair(rng, len(X), 6, 6, Q)
    _, fl = t.flowtree(mu, mm, nu, nm, Q=Q)
    a, b = mm / 2.0 ** Q, nm / 2.0 ** Q
    gX, _, _ = oracle.frozen_grad(X, mu, nu, fl, a, b)
    X64 = X.astype(np.float64)
    h = 1e-3
    pts = np.unique(np.concatenate([mu, nu]))
    for p in pts:
        for i in range(X.shape[1]):
            Xp = X64.copy(); Xp[p, i] += h
            Xm = X64.copy(); Xm[p, i] -= h
            fd = (oracle.frozen_cost(Xp, mu, nu, fl, a, b) - oracle.frozen_cost(Xm, mu, nu, fl, a, b)) / (2 * h)
            assert fd == pytest.approx(gX[p, i], abs=2e-6)
    others = np.setdiff1d(np.arange(len(X)), pts)
    assert np.abs(gX[others]).max() == 0.0


@pytest.mark.parametrize("seed", range(6))
def test_grad_weights_fd(seed):
    rng, X, t = world(seed)
    Q = 16
    mu, mm, nu, nm = pair(rng, len(X), 5, 8, Q)
    _, fl = t.flowtree(mu, mm, nu, nm, Q=Q)
    a, b = mm / 2.0 ** Q, nm / 2.0 ** Q
    _, ga, gb = oracle.frozen_grad(X, mu, nu, fl, a, b)
    h = 1e-3
    for w, g, which in ((a, ga, 0), (b, gb, 1)):
        for i in range(len(w)):
            wp = w.copy(); wp[i] += h
            wm = w.copy(); wm[i] -= h
            args_p = (wp, b) if which == 0 else (a, wp)
            args_m = (wm, b) if which == 0 else (a, wm)
            fd = (oracle.frozen_cost(X, mu, nu, fl, *args_p) - oracle.frozen_cost(X, mu, nu, fl, *args_m)) / (2 * h)
            assert fd == pytest.approx(g[i], rel=1e-9, abs=1e-12)


def test_grad_single_pair_closed_form():
    rng, X, t = world(1)
    Q = 8
    for _ in range(20):
        x, y = map(int, rng.choice(len(X), 2, replace=False))
        m = np.array([1 << Q], np.uint32)
        _, fl = t.flowtree([x], m, [y], m, Q=Q)
        gX, ga, gb = oracle.frozen_grad(X, np.array([x]), np.array([y]), fl, [1.0], [1.0])
        diff = X[x].astype(float) - X[y]
        D = np.linalg.norm(diff)
        assert np.allclose(gX[x], diff / D, rtol=1e-13)
        assert np.allclose(gX[y], -diff / D, rtol=1e-13)
        # one emission bound on both sides: the whole adjoint goes to mu
        assert ga[0] == pytest.approx(D, rel=1e-13) and gb[0] == 0.0


@pytest.mark.parametrize("seed", range(10))
def test_integer_unit_move_through_real_greedy(seed):
    rng, X, t = world(seed)
    Q = 20
    mu, mm, nu, nm = pair(rng, len(X), 6, 6, Q)
    c0, fl = t.flowtree(mu, mm, nu, nm, Q=Q)
    _, ga, gb = oracle.frozen_grad(X, mu, nu, fl, mm / 2.0 ** Q, nm / 2.0 ** Q)
    pattern = list(zip(fl["mu"].tolist(), fl["nu"].tolist(), fl["bind"].tolist()))
    checked = 0
    for side in (0, 1):
        m = (mm if side == 0 else nm).astype(np.int64)
        g = ga if side == 0 else gb
        for i in range(len(m)):
            for j in range(len(m)):
                if i == j or m[j] < 3:
                    continue
                m2 = m.copy(); m2[i] += 1; m2[j] -= 1
                args = (mu, m2, nu, nm) if side == 0 else (mu, mm, nu, m2)
                c1, fl1 = t.flowtree(*args, Q=Q)
                p1 = list(zip(fl1["mu"].tolist(), fl1["nu"].tolist(), fl1["bind"].tolist()))
                if p1 != pattern:
                    continue
                assert (c1 - c0) * 2.0 ** Q == pytest.approx(g[i] - g[j], rel=1e-6, abs=1e-9)
                checked += 1
    assert checked > 0
