"""Pins of the per-inner-sample regression rows (Section 3.2: the samples of I = M x n_b with
the default indicators as inputs).

  * the draw average of the labels is the inner-average target T; the indicators of draw l
    switch on at its default date and their increments add up to the default counts;
  * for one counterparty, the per-sample loss of any predictor that puts 0 on the dead samples
    equals the grouped alive-row loss (weights A / n_b) plus a predictor-free term, so the
    literal rows and the grouped form train the same alive branch;
  * the label of every sample matches eq:CVA_portfolio written out as a double loop over dates
    and counterparties on a tiny case.
"""
import numpy as np

import workloads as wl
from oracle import inner, model


def case(w):
    paths = np.arange(w.M)
    o = model.simulate_outer(w, paths)
    mt = model.mtm(w, o)
    u = inner.inner_draws(w, paths)
    js = inner.default_dates(o.Lam, u)
    xi = inner.pathwise_loss(o.I, mt, w.market.lgd, js)
    return o, mt, js, xi, model.features(w, o)


def test_rows_average_to_targets_and_count_defaults():
    w = wl.small_multi(M=40, n_b=6)
    o, mt, js, xi, F = case(w)
    X, Y = inner.sample_rows(F, xi, js)
    n, d, C, P = w.grid.n_dates, F.shape[1], w.market.n_cpty, w.M
    T = inner.targets(xi)
    assert np.allclose(Y.reshape(n + 1, w.n_b, P).mean(axis=1), T, rtol=1e-13, atol=0)
    ind = X[:, d:, :]                                        # [n+1, C, n_b P]
    assert np.all(ind[0] == 0)                               # nobody defaults at t_0
    inc = np.diff(ind, axis=0).reshape(n, C, w.n_b, P).sum(axis=2)
    assert np.array_equal(inc, inner.default_counts(js, n)[1:])
    for l in range(w.n_b):                                   # the market inputs are the path's
        assert np.array_equal(X[:, :d, l * P:(l + 1) * P], F)


def test_one_counterparty_rows_equal_the_grouped_form():
    w = wl.plain_fp64().with_(M=64, n_b=32)
    o, mt, js, xi, F = case(w)
    X, Y = inner.sample_rows(F, xi, js)
    t, wt = inner.alive_targets(xi, js)
    n1, P = Y.shape[0], w.M
    rng = np.random.default_rng(2)
    phi_alive = rng.uniform(0.0, 2.0 * Y.max(), (n1, P))     # any predictor of the alive branch
    dead = X[:, -1, :] == 1.0
    pred = np.where(dead, 0.0, np.tile(phi_alive, (1, w.n_b)))
    per_sample = ((pred - Y) ** 2).reshape(n1, w.n_b, P).sum(axis=1)
    grouped = w.n_b * wt * (phi_alive - t) ** 2
    const = per_sample - grouped
    phi2 = rng.uniform(0.0, 2.0 * Y.max(), (n1, P))
    pred2 = np.where(dead, 0.0, np.tile(phi2, (1, w.n_b)))
    per_sample2 = ((pred2 - Y) ** 2).reshape(n1, w.n_b, P).sum(axis=1)
    assert np.allclose(per_sample2 - w.n_b * wt * (phi2 - t) ** 2, const, rtol=1e-9,
                       atol=1e-9 * float(per_sample.max()))


def test_labels_follow_the_loss_definition_on_a_tiny_case():
    w = wl.tiny(M=3, n_b=5)
    o, mt, js, xi, F = case(w)
    X, Y = inner.sample_rows(F, xi, js)
    n, P, C = w.grid.n_dates, w.M, w.market.n_cpty
    for k in range(P):
        for l in range(w.n_b):
            for i in range(n + 1):
                s = 0.0
                for c in range(C):
                    for j in range(i, n):                    # default in (t_j, t_{j+1}]
                        if js[k, l, c] == j + 1:
                            s += (np.exp(o.I[i, k] - o.I[j + 1, k]) * w.market.lgd[c]
                                  * max(mt[j + 1, k, c], 0.0))
                assert abs(Y[i, l * P + k] - s) <= 1e-12 * max(1.0, abs(s))
