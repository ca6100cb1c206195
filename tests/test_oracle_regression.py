"""Pins of the oracle's neural regression (BaseAlg / Backward learning), CPU."""
import numpy as np

import workloads as wl
from oracle import regression as rg


def rand_problem(M=64, d=3, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((M, d))
    y = np.maximum(X @ rng.standard_normal(d), 0.0) + 0.1 * rng.standard_normal(M) + 0.5
    return X, y


def test_init_is_deterministic_and_bounded():
    a = rg.init_net(5, 2, 7, seed=3)
    b = rg.init_net(5, 2, 7, seed=3)
    c = rg.init_net(5, 2, 7, seed=4)
    for wa, wb, wc, (fo, fi) in zip(a.W, b.W, c.W, rg.layer_shapes(5, 2, 7)):
        assert wa.shape == (fo, fi)
        assert np.array_equal(wa, wb)
        assert not np.array_equal(wa, wc)
        assert np.all(np.abs(wa) < 1.0 / np.sqrt(fi))
    # the draws are close to uniform on the bound
    big = rg.init_net(64, 1, 256, seed=0).W[0] * 8.0
    assert abs(big.mean()) < 0.02 and abs(big.var() - 1.0 / 3.0) < 0.02


def test_backprop_matches_central_differences():
    X, y = rand_problem()
    net = rg.init_net(3, 2, 5, seed=1)
    net.mu = 0.2
    net.b = [np.linspace(-0.3, 0.3, v.size) for v in net.b]
    for pos in (0, 1):
        gW, gb, gmu = rg.grads(net, X, y, pos)
        h = 1e-6
        for l in range(len(net.W)):
            for idx in [(0, 0), (net.W[l].shape[0] - 1, net.W[l].shape[1] - 1)]:
                up, dn = net.copy(), net.copy()
                up.W[l][idx] += h
                dn.W[l][idx] -= h
                fd = (rg.loss(up, X, y, pos) - rg.loss(dn, X, y, pos)) / (2 * h)
                assert np.isclose(gW[l][idx], fd, rtol=1e-6, atol=1e-9), (pos, l, idx)
            up, dn = net.copy(), net.copy()
            up.b[l][0] += h
            dn.b[l][0] -= h
            fd = (rg.loss(up, X, y, pos) - rg.loss(dn, X, y, pos)) / (2 * h)
            assert np.isclose(gb[l][0], fd, rtol=1e-6, atol=1e-9)
        up, dn = net.copy(), net.copy()
        up.mu += h
        dn.mu -= h
        fd = (rg.loss(up, X, y, pos) - rg.loss(dn, X, y, pos)) / (2 * h)
        assert np.isclose(gmu, fd, rtol=1e-6, atol=1e-9)


def test_first_adam_step_moves_by_signed_lr():
    """With fresh moments, bias correction makes the first step -lr g / (|g| + eps)."""
    X, y = rand_problem()
    net = rg.init_net(3, 1, 4, seed=2)
    before = net.copy()
    gW, gb, gmu = rg.grads(net, X, y, 0)
    opt = rg.Adam(net, lr=1e-2)
    opt.step(net, gW, gb, gmu)
    for l in range(len(net.W)):
        step = net.W[l] - before.W[l]
        assert np.allclose(step, -1e-2 * gW[l] / (np.abs(gW[l]) + 1e-8), rtol=1e-12, atol=1e-15)
    assert np.isclose(net.mu - before.mu, -1e-2 * gmu / (abs(gmu) + 1e-8), rtol=1e-12)


def test_output_refit_is_stationary():
    """After the closed-form refit, the gradient of the ridge-penalised pos=0 loss in
    (W^{h+1}, b^{h+1}) vanishes, and with the ridge switched off the refit is the OLS fit."""
    X, y = rand_problem(M=200)
    net = rg.init_net(3, 2, 6, seed=5)
    net.mu = 0.3
    rg.refit_output_layer(net, X, y)
    gW, gb, _ = rg.grads(net, X, y, 0)
    acts, _, _ = rg.forward(net, X)
    H = np.concatenate([acts[-1], np.ones((X.shape[0], 1))], axis=1)
    G = H.T @ H
    lam = rg.REFIT_RIDGE * np.trace(G) / G.shape[0]
    # d/dw [ (1/M) |H w + mu - y|^2 + (lam/M) |w|^2 ] = grads + 2 lam w / M
    w = np.concatenate([net.W[-1][0], net.b[-1]])
    pen = 2.0 * lam * w / X.shape[0]
    assert np.max(np.abs(gW[-1][0] + pen[:-1])) < 1e-10
    assert abs(gb[-1][0] + pen[-1]) < 1e-10
    old = rg.REFIT_RIDGE
    try:
        rg.REFIT_RIDGE = 0.0
        rg.refit_output_layer(net, X, y)
    finally:
        rg.REFIT_RIDGE = old
    sol, *_ = np.linalg.lstsq(H, y - net.mu, rcond=None)
    assert np.allclose(np.concatenate([net.W[-1][0], net.b[-1]]), sol, rtol=1e-8, atol=1e-10)


def test_linear_network_converges_to_ols():
    """h = 0 is linear regression (e:forw): Adam on the pos=0 loss reaches the OLS fit."""
    X, y = rand_problem(M=128, d=3, seed=7)
    net = rg.init_net(3, 0, 1, seed=0)
    opt = rg.Adam(net, lr=2e-2)
    for _ in range(6000):
        opt.step(net, *rg.grads(net, X, y, 0))
    A = np.concatenate([X, np.ones((X.shape[0], 1))], axis=1)
    coef = np.linalg.solve(A.T @ A, A.T @ y)          # normal equations
    assert np.allclose(rg.predict_scaled(net, X, 0), A @ coef, atol=1e-6)


def test_base_alg_keeps_best_parameters():
    X, y = rand_problem(M=256, seed=9)
    net = rg.init_net(3, 2, 8, seed=0)
    res = rg.base_alg(net, X, y, epochs=6, batch=32)
    assert len(res.losses) == 6
    assert np.isclose(res.best_loss, min(res.losses))
    assert np.isclose(rg.loss(res.net, X, y, 1), res.best_loss)
    assert res.best_loss < rg.loss(rg.init_net(3, 2, 8, seed=0), X, y, 1)


def test_backward_learning_warm_start_and_empty_dates():
    w = wl.tiny()
    rng = np.random.default_rng(0)
    n = 4
    feats = rng.standard_normal((n + 1, 3, 32))
    T = np.abs(rng.standard_normal((n + 1, 32)))
    T[n] = 0.0                                  # nothing left to lose at the horizon
    cfg = wl.MLPConfig(hidden=1, width=4, epochs=2, n_batches=2)
    out = rg.backward_learning(feats, T, cfg, seed=0)
    assert sorted(out) == [1, 2, 3, 4]
    assert not out[4].trained
    assert np.all(rg.predict(out[4], feats[4].T) == 0.0)
    assert out[3].trained
    p3 = rg.predict(out[3], feats[3].T)
    assert np.all(p3 >= out[3].net.mu * out[3].scaling.y_scale - 1e-12)
