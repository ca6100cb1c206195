"""Pins of the grouped per-inner-sample regression data (one counterparty) and of the weighted
regression (Section 3.2 with X the default indicator; Algorithm 1 with row weights).

  * a draw whose client has defaulted by t_i has xi_i = 0 exactly (nothing is left to lose);
  * the alive group's sum of squares over draws equals A (phi - target)^2 plus a term free of
    phi, for any phi: the weighted row reproduces the paper's per-sample loss;
  * weight x target = the inner average over all draws (the dead draws add nothing);
  * with many draws the alive target approaches the survival-conditioned mean
    mu_i / exp(-Lambda_i) of the exact conditional moments (z-test);
  * weighted regression: integer weights equal duplicated rows (loss, full-batch gradient,
    refit); unit weights equal the unweighted fit up to summation order.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import inner, model, pipeline
from oracle import regression as org


@pytest.fixture(scope="module")
def plain():
    w = wl.plain_fp64().with_(M=256, n_b=64)
    paths = np.arange(w.M)
    o = model.simulate_outer(w, paths)
    mt = model.mtm(w, o)
    u = inner.inner_draws(w, paths)
    js = inner.default_dates(o.Lam, u)
    xi = inner.pathwise_loss(o.I, mt, w.market.lgd, js)
    return w, o, mt, js, xi


def test_dead_draws_carry_no_loss(plain):
    w, o, mt, js, xi = plain
    n = w.grid.n_dates
    dead = js[None, :, :, 0] <= np.arange(n + 1)[:, None, None]
    assert dead.any() and np.all(xi[dead] == 0.0)


def test_alive_group_reproduces_the_per_sample_loss(plain):
    w, o, mt, js, xi = plain
    t, wt = inner.alive_targets(xi, js)
    n_b = xi.shape[2]
    A = np.rint(wt * n_b)
    rng = np.random.default_rng(3)
    alive = js[None, :, :, 0] > np.arange(xi.shape[0])[:, None, None]
    for phi in (rng.uniform(0, 2 * xi.max(), t.shape), np.zeros(t.shape)):
        lhs = np.where(alive, (phi[:, :, None] - xi) ** 2, 0.0).sum(axis=2)
        const = np.where(alive, (xi - t[:, :, None]) ** 2, 0.0).sum(axis=2)
        rhs = A * (phi - t) ** 2 + const
        assert np.allclose(lhs, rhs, rtol=1e-10, atol=1e-12 * float(lhs.max()))
    # weight x target is the inner average over all draws
    assert np.allclose(wt * t, inner.targets(xi), rtol=1e-12, atol=0.0)
    # at t_0 everybody is alive
    assert np.all(wt[0] == 1.0) and np.array_equal(t[0], inner.targets(xi)[0])


def test_alive_target_is_the_survival_conditioned_mean():
    w = wl.plain_fp64().with_(M=128, n_b=4096)
    r = pipeline.simulate(w, with_moments=True, with_alive=True)
    n = w.grid.n_dates
    S = np.exp(-np.transpose(r["Lam"], (0, 2, 1))[:, :, 0])          # survival given the path
    mean_alive = r["mu"] / S
    m2_alive = (r["var"] + r["mu"] ** 2) / S
    var_alive = np.maximum(m2_alive - mean_alive ** 2, 0.0)
    A = r["W_alive"] * w.n_b
    i = np.arange(1, n)
    num = (r["T_alive"][i] - mean_alive[i]).sum(axis=1)
    den = np.sqrt((var_alive[i] / np.maximum(A[i], 1)).sum(axis=1))
    live = den > 0
    assert np.all(np.abs(num[~live]) <= 1e-9 * np.abs(mean_alive).max())
    z = num[live] / den[live]
    print(f"  per-date path sums: max |z| = {np.abs(z).max():.2f} over {live.sum()} dates")
    assert live.sum() > n // 2 and np.abs(z).max() < 5.0


def test_integer_weights_equal_duplicated_rows():
    rng = np.random.default_rng(5)
    M, d = 40, 3
    X = rng.standard_normal((M, d))
    y = np.abs(rng.standard_normal(M))
    w = rng.integers(0, 4, M).astype(np.float64)
    Xd = np.repeat(X, w.astype(int), axis=0)
    yd = np.repeat(y, w.astype(int))
    net = org.init_net(d, 2, 8, seed=1)
    for pos in (0, 1):
        # (1/M) sum w r^2 = (M_dup / M) (1/M_dup) sum over the duplicated rows
        assert org.loss(net, X, y, pos, w) == pytest.approx(
            org.loss(net, Xd, yd, pos) * Xd.shape[0] / M, rel=1e-12)
        gW, gb, gmu = org.grads(net, X, y, pos, w)
        dW, db, dmu = org.grads(net, Xd, yd, pos)
        f = Xd.shape[0] / M
        for a, b in zip(gW + gb, dW + db):
            assert np.allclose(a, f * b, rtol=1e-10, atol=1e-14)
        assert gmu == pytest.approx(f * dmu, rel=1e-10)
    n1, n2 = net.copy(), net.copy()
    org.refit_output_layer(n1, X, y, w)
    org.refit_output_layer(n2, Xd, yd)
    assert np.allclose(n1.W[-1], n2.W[-1], rtol=1e-9) and np.allclose(n1.b[-1], n2.b[-1], rtol=1e-9)


def test_unit_weights_equal_the_unweighted_fit():
    w = wl.small_multi(M=256)
    r = pipeline.simulate(w)
    mlp = wl.MLPConfig(hidden=1, width=32, epochs=4, batch=64)
    a = org.independent_fits(r["features"], r["T"], mlp, w.seed, [5])
    b = org.independent_fits(r["features"], r["T"], mlp, w.seed, [5], W=np.ones_like(r["T"]))
    # equal up to the summation order of the refit's Gram product
    assert np.allclose(a[5].losses, b[5].losses, rtol=1e-9, atol=0.0)
    assert all(np.allclose(x, y, rtol=1e-7, atol=1e-12) for x, y in zip(a[5].net.W, b[5].net.W))
