"""Pins of the oracle's inner default draws, pathwise loss and targets (CPU)."""
import numpy as np
import pytest

import workloads as wl
from oracle import closed_forms as cf
from oracle import inner, model, pipeline


def test_default_rule_literal_cases():
    # n = 3 dates, one path, one counterparty; Lambda = 0, 0.1, 0.2, 0.5
    Lam = np.array([0.0, 0.1, 0.2, 0.5])[:, None, None]
    eps = np.array([0.05, 0.0999, 0.15, 0.2001, 0.49, 0.5001, 3.0])
    u = np.exp(-eps)[None, :, None]
    js = inner.default_dates(Lam, u)[0, :, 0]
    # eps < 0.1 -> date 1, < 0.2 -> 2, < 0.5 -> 3, beyond the horizon -> none (n + 1 = 4)
    assert list(js) == [1, 1, 2, 3, 3, 4, 4]
    # equality counts as a default: a threshold exactly equal to Lambda_j defaults at j
    Lam2 = np.array([0.0, 0.25, 0.5, 1.0])[:, None, None]
    u2 = np.array([0.5])[None, :, None]          # -log(0.5) vs Lambda = 0.5 is not exact;
    e = -np.log(u2)
    Lam2[2] = e[0, 0, 0]                          # so set Lambda_2 to the very value of eps
    assert inner.default_dates(Lam2, u2)[0, 0, 0] == 2


def brute_force_xi(I, mtm_c, lgd, js):
    """xi_i by the direct double sum of the loss formula (no recursion)."""
    n = I.shape[0] - 1
    P, n_b, C = js.shape
    beta = np.exp(-I)
    xi = np.zeros((n + 1, P, n_b))
    for i in range(n + 1):
        for k in range(P):
            for l in range(n_b):
                tot = 0.0
                for c in range(C):
                    for j in range(i, n):
                        if js[k, l, c] == j + 1:
                            tot += beta[j + 1, k] / beta[i, k] * lgd[c] * max(mtm_c[j + 1, k, c], 0.0)
                xi[i, k, l] = tot
    return xi


def test_brute_force_tiny():
    w = wl.tiny()
    paths = np.arange(w.M)
    o = model.simulate_outer(w, paths)
    mt = model.mtm(w, o)
    u = inner.inner_draws(w, paths)
    js = inner.default_dates(o.Lam, u)
    xi = inner.pathwise_loss(o.I, mt, w.market.lgd, js)
    ref = brute_force_xi(o.I, mt, w.market.lgd, js)
    assert np.allclose(xi, ref, rtol=1e-14, atol=0)
    # make defaults certain to exercise the sums: huge intensities
    Lam_big = o.Lam * 1e3
    js2 = inner.default_dates(Lam_big, u)
    assert np.all(js2 <= w.grid.n_dates)
    xi2 = inner.pathwise_loss(o.I, mt, w.market.lgd, js2)
    assert np.allclose(xi2, brute_force_xi(o.I, mt, w.market.lgd, js2), rtol=1e-14, atol=0)


@pytest.fixture(scope="module")
def plain_run():
    w = wl.plain_fp64().with_(M=2048, n_b=64)
    r = pipeline.simulate(w, with_moments=True)
    return w, r


def test_target_matches_exact_conditional_mean(plain_run):
    """(T - mu)/(sigma/sqrt(n_b)) is N(0,1) across paths at every date."""
    w, r = plain_run
    for i in (0, 10, 25, 40):
        sd = np.sqrt(r["var"][i] / w.n_b)
        ok = sd > 0
        z = (r["T"][i][ok] - r["mu"][i][ok]) / sd[ok]
        assert abs(z.mean()) < 5.0 / np.sqrt(z.size), i
        assert abs(z.var() - 1.0) < 0.2, i


def test_alive_frequency_matches_cir_survival(plain_run):
    w, r = plain_run
    m = w.market
    n = w.grid.n_dates
    for i in (5, 25, 50):
        dead = r["cnt"][1:i + 1].sum(axis=0)[0] / w.n_b
        alive = 1.0 - dead
        S = cf.cir_survival(m.kappa[0], m.theta[0], m.nu[0], m.lambda0[0], i * w.grid.horizon / n)
        assert abs(alive.mean() - S) < 5 * alive.std() / np.sqrt(alive.size) + 5e-4


def test_unbiased_against_single_draw():
    """Paired with n_b = 1 (its draw is the first of the n_b), the mean difference is 0."""
    w = wl.plain_fp64().with_(M=4096)
    t1 = pipeline.simulate(w, n_b=1)["T"]
    t16 = pipeline.simulate(w, n_b=16)["T"]
    for i in (0, 10, 30):
        d = t16[i] - t1[i]
        assert abs(d.mean()) < 5 * d.std() / np.sqrt(d.size)


def test_variance_falls_as_one_over_nb():
    """Var_k T_i = R_i + Q_i / n_b with R = Var(mu), Q = E[var] from the exact moments."""
    w = wl.plain_fp64().with_(M=4096)
    base = pipeline.simulate(w, n_b=1, with_moments=True)
    for i in (0, 20):
        R = base["mu"][i].var()
        Q = base["var"][i].mean()
        for n_b in (1, 8, 64):
            T = pipeline.simulate(w, n_b=n_b)["T"][i]
            expect = R + Q / n_b
            # standard error of a sample variance from the sample's fourth moment
            d = T - T.mean()
            se = np.sqrt(((d ** 4).mean() - d.var() ** 2) / T.size)
            assert abs(T.var() - expect) < 5 * se, (i, n_b, T.var(), expect)
        assert Q > 5 * R      # the inner (default) part dominates at n_b = 1 here


def test_independence_factorisation():
    """Market and credit are independent here, so
    CVA_0 = sum_j LGD E[beta_j (MtM_j)^+] (S(t_{j-1}) - S(t_j)) up to Euler and MC error."""
    w = wl.plain_fp64().with_(M=2048)
    r = pipeline.simulate(w, with_moments=True)
    m = w.market
    n = w.grid.n_dates
    beta = np.exp(-r["I"])
    e_pos = (beta * np.maximum(r["MtM"][:, 0, :], 0.0)).mean(axis=1)
    t = np.arange(n + 1) * w.grid.horizon / n
    S = cf.cir_survival(m.kappa[0], m.theta[0], m.nu[0], m.lambda0[0], t)
    ref = m.lgd[0] * np.sum(e_pos[1:] * (S[:-1] - S[1:]))
    mu0 = r["mu"][0]
    # the smoothed estimator has small variance: 5 s.e. plus an Euler/cross-term allowance
    assert abs(mu0.mean() - ref) < 5 * mu0.std() / np.sqrt(mu0.size) + 0.02 * ref
    T0 = r["T"][0]
    assert abs(T0.mean() - ref) < 5 * T0.std() / np.sqrt(T0.size) + 0.02 * ref


def test_uneven_oversimulation_prefix():
    """A path simulated with n_b' draws inside an uneven sweep equals a uniform run at n_b'."""
    w = wl.oversim_sweep(M=256, levels=(1, 8))
    nbp = np.repeat(w.extra["n_b_per_block"], 64)[:w.M]
    r = pipeline.simulate(w, n_b_per_path=nbp)
    r8 = pipeline.simulate(w, n_b=8)
    sel = nbp == 8
    assert np.array_equal(r["T"][:, sel], r8["T"][:, sel])
