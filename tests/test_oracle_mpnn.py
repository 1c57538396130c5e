"""Pins of the CPU FP64 surrogate reference: the analytic gradient against
central finite differences, Adam against its closed form on a quadratic,
and the features against brute-force loops."""
import numpy as np

import workloads as W
from oracle import mpnn as M


def _setup(seed=0):
    g = W.grid2d(7, 6, seed=seed, wdist=("lognormal", 0.0, 1.0))
    import oracle

    rng = np.random.default_rng(seed)
    tree = oracle.max_spanning_forest(g.n, g.u, g.v, g.w)[0].astype(bool)
    xc = rng.standard_normal((g.n, 4))
    cand = np.nonzero(~tree)[0]
    nf, ef = M.raw_features(g.n, g.u, g.v, g.w, tree, xc, cand)
    norm = np.concatenate([nf.mean(0), 1 / (nf.std(0) + 1e-3), ef.mean(0), 1 / (ef.std(0) + 1e-3)])
    X, E = M.standardise(nf, ef, norm)
    A, d = M.norm_adjacency(g.n, g.u, g.v, g.w)
    y = rng.standard_normal(cand.shape[0])
    theta = M.init_params(seed + 1) + 0.01     # nonzero biases: every ReLU branch is exercised
    return g, A, d, X, E, cand, y, theta, tree, xc


def test_param_count():
    assert M.n_params() == 4865


def test_gradient_matches_finite_differences():
    g, A, d, X, E, cand, y, theta, _, _ = _setup()
    yhat, cache = M.forward(theta, A, d, X, g.u, g.v, cand, E)
    grad = M.backward(theta, A, d, X, y, yhat, cache)
    rng = np.random.default_rng(5)
    idx = rng.choice(theta.shape[0], 200, replace=False)
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        lp = M.loss(M.forward(tp, A, d, X, g.u, g.v, cand, E)[0], y)
        lm = M.loss(M.forward(tm, A, d, X, g.u, g.v, cand, E)[0], y)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, grad[i])


def test_adam_on_quadratic():
    # Adam with lr small on f = |theta|^2 / 2: the first step moves every coordinate by -lr (bias corrected)
    theta = np.array([3.0, -2.0, 0.5])
    m = np.zeros(3)
    v = np.zeros(3)
    t1, m, v = M.adam_step(theta, theta.copy(), m, v, 1, lr=1e-3)
    assert np.allclose(t1, theta - 1e-3 * np.sign(theta), rtol=0, atol=1e-10)


def test_features_brute_force():
    g, _, _, _, _, cand, _, _, tree, xc = _setup(3)
    nf, ef = M.raw_features(g.n, g.u, g.v, g.w, tree, xc, cand)
    for p in range(g.n):
        inc = [e for e in range(g.m) if p in (g.u[e], g.v[e])]
        other = [int(g.v[e] if g.u[e] == p else g.u[e]) for e in inc]
        dG = sum(g.w[e] for e in inc)
        tin = [e for e in inc if tree[e]]
        dT = sum(g.w[e] for e in tin)
        eG = sum(g.w[e] * np.sum((xc[p] - xc[o]) ** 2) for e, o in zip(inc, other))
        assert np.isclose(nf[p, 1], np.log(dG)) and np.isclose(nf[p, 2], np.log(dT))
        assert np.isclose(nf[p, 3], np.log(len(inc))) and np.isclose(nf[p, 4], np.log(len(tin)))
        assert np.isclose(nf[p, 6], np.log(eG / dG))
    e = cand[0]
    assert np.isclose(ef[0, 1], np.log(g.w[e] * np.sum((xc[g.u[e]] - xc[g.v[e]]) ** 2)))
