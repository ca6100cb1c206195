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


def _hidden(net, X):
    acts, _, _ = rg.forward(net, X)
    return np.concatenate([acts[-1], np.ones((X.shape[0], 1))], axis=1)


def test_output_refit_solves_the_least_squares_problem():
    """Algorithm 1's closed-form refit is the argmin of the pos = 0 loss over the output layer:
    at the solution the loss gradient in (W^{h+1}, b^{h+1}) vanishes (normal equations), and no
    perturbation of the output layer lowers the loss."""
    X, y = rand_problem(M=200)
    net = rg.init_net(3, 2, 6, seed=5)
    net.mu = 0.3
    rg.refit_output_layer(net, X, y)
    gW, gb, _ = rg.grads(net, X, y, 0)
    H = _hidden(net, X)
    scale = np.abs(H).max() * np.abs(y - net.mu).max()
    assert np.max(np.abs(gW[-1][0])) < 1e-12 * scale
    assert abs(gb[-1][0]) < 1e-12 * scale
    L0 = rg.loss(net, X, y, 0)
    rng = np.random.default_rng(1)
    for _ in range(200):
        p = net.copy()
        p.W[-1] = p.W[-1] + 1e-3 * rng.standard_normal(p.W[-1].shape)
        p.b[-1] = p.b[-1] + 1e-3 * rng.standard_normal(1)
        assert rg.loss(p, X, y, 0) >= L0


def test_output_refit_recovers_an_exact_linear_target():
    """Targets exactly affine in the hidden features: the refit returns those coefficients."""
    X, _ = rand_problem(M=300, seed=4)
    net = rg.init_net(3, 2, 6, seed=8)
    net.b = [np.linspace(0.2, 0.6, v.size) for v in net.b]      # every unit active somewhere
    net.mu = -0.1
    H = _hidden(net, X)
    assert np.linalg.matrix_rank(H) == H.shape[1]
    w_true = np.array([0.5, -1.25, 2.0, 0.0, 0.75, -0.3, 0.05])
    y = H @ w_true + net.mu
    rg.refit_output_layer(net, X, y)
    got = np.concatenate([net.W[-1][0], net.b[-1]])
    assert np.allclose(got, w_true, rtol=0, atol=1e-10)


def test_output_refit_minimum_norm_on_dead_and_duplicated_units():
    """Rank-deficient hidden features: a dead ReLU unit (all-zero column) gets weight 0 and two
    identical units share their weight equally (the minimum-norm least-squares solution), while
    the fitted values stay those of the full-rank problem without the redundant columns."""
    X, y = rand_problem(M=250, seed=6)
    net = rg.init_net(3, 2, 6, seed=9)
    net.b[1][2] = -1e3                       # unit 2 of the last hidden layer never fires
    net.W[1][4] = net.W[1][1]                # unit 4 duplicates unit 1
    net.b[1][4] = net.b[1][1]
    net.mu = 0.1
    rg.refit_output_layer(net, X, y)
    w = net.W[-1][0]
    H = _hidden(net, X)
    assert np.all(H[:, 2] == 0.0)
    assert abs(w[2]) < 1e-12
    assert abs(w[4] - w[1]) < 1e-10 * max(1.0, abs(w[1]))
    keep = [0, 1, 3, 5, 6]                   # independent columns (bias last)
    Hk = H[:, keep]
    coef = np.linalg.solve(Hk.T @ Hk, Hk.T @ (y - net.mu))
    assert np.allclose(H @ np.concatenate([w, net.b[-1]]), Hk @ coef, rtol=0, atol=1e-10)


def _guarded_cholesky_fit(H, r, guard=1e-12):
    """The library's refit solve written out in NumPy: normal equations of [H, 1], a Cholesky
    factorisation in which a column whose diagonal is zero, or whose pivot falls to
    guard x its diagonal, is dropped (weight 0); the rest solved by the two triangular solves."""
    G = H.T @ H
    rhs = H.T @ r
    n = G.shape[0]
    Lm = G.copy()
    drop = np.zeros(n, dtype=bool)
    for k in range(n):
        p = Lm[k, k]
        if G[k, k] == 0.0 or p <= guard * G[k, k]:
            drop[k] = True
            Lm[k:, k] = 0.0
            Lm[k, k] = 1.0
            continue
        Lm[k, k] = np.sqrt(p)
        Lm[k + 1:, k] /= Lm[k, k]
        Lm[k + 1:, k + 1:] -= np.outer(Lm[k + 1:, k], Lm[k + 1:, k])
    L = np.tril(Lm)
    z = np.zeros(n)
    for i in range(n):
        z[i] = 0.0 if drop[i] else (rhs[i] - L[i, :i] @ z[:i]) / L[i, i]
    x = np.zeros(n)
    for i in range(n - 1, -1, -1):
        x[i] = 0.0 if drop[i] else (z[i] - L[i + 1:, i] @ x[i + 1:]) / L[i, i]
    return x, drop


def test_library_refit_rule_gives_the_least_squares_fitted_values():
    """The GPU solves the refit by a Cholesky factorisation of the normal equations that drops
    zero and dependent columns (pivot <= 1e-12 x diagonal).  On the hidden features of a
    three-layer, 128-unit network with dead units and nearly collinear columns, its fitted
    values equal the oracle's minimum-norm least squares to 1e-9 relative."""
    rng = np.random.default_rng(11)
    M, d = 4096, 29
    X = rng.standard_normal((M, d))
    y = np.log1p(np.exp(X @ rng.standard_normal(d) / np.sqrt(d))) + 0.1 * rng.standard_normal(M)
    net = rg.init_net(d, 3, 128, seed=2)
    net.b[2][:10] = -50.0                     # ten dead units in the last hidden layer
    net.W[2][20] = net.W[2][21] * (1 + 1e-13)  # an (almost) exactly duplicated unit
    net.b[2][20] = net.b[2][21] * (1 + 1e-13)
    H = _hidden(net, X)
    r = y - 0.05
    ref = net.copy()
    ref.mu = 0.05
    rg.refit_output_layer(ref, X, y)
    f_ref = H @ np.concatenate([ref.W[-1][0], ref.b[-1]])
    x, drop = _guarded_cholesky_fit(H, r)
    assert drop[:10].all() and drop.sum() >= 11
    f = H @ x
    assert np.linalg.norm(f - f_ref) <= 1e-9 * np.linalg.norm(f_ref)


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
