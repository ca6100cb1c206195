"""Pins of the oracle's outer simulation and pricing against closed forms (CPU).

Statistical checks use fixed seeds and |z| <= 5 bounds, so they are deterministic.
"""
import numpy as np
import pytest
from scipy import integrate

import workloads as wl
from oracle import closed_forms as cf
from oracle import model


def two_ccy_workload(M=16384, n_dates=10, n_sub=40, rho=0.6, seed=3, sigma_fx=0.25):
    corr = np.array([[1.0, 0.2, 0.1], [0.2, 1.0, rho], [0.1, rho, 1.0]])
    mkt = wl.Market(a=np.array([0.1, 0.15]), b=np.array([0.02, 0.03]),
                    sigma_r=np.array([0.01, 0.012]), r0=np.array([0.02, 0.025]),
                    sigma_fx=np.array([sigma_fx]), fx0=np.array([1.3]), corr=corr,
                    kappa=np.array([0.5]), theta=np.array([0.02]), nu=np.array([0.1]),
                    lambda0=np.array([0.02]), lgd=np.array([0.6]))
    book = wl.Portfolio(ccy=np.array([0, 1, 1], np.int32), cpty=np.zeros(3, np.int32),
                        maturity=np.array([4, 3, 5], np.int32),
                        notional=np.array([1.0, 1.0, 1.0]),
                        spread_bp=np.array([0.0, 30.0, -20.0]),
                        payer=np.array([1, -1, 1], np.int32))
    return wl.Workload(name="two_ccy", market=mkt, portfolio=book,
                       grid=wl.Grid(10.0, n_dates, n_sub), M=M, n_b=1, seed=seed)


# ------------------------------------------------------------------ closed forms themselves
def test_vasicek_zc_matches_gaussian_integral():
    """exp(-m + v/2) with m, v the mean/variance of int_0^T r by quadrature of OU moments."""
    a, b, s, r0 = 0.13, 0.03, 0.015, 0.01
    for T in (0.5, 3.0, 10.0):
        m = integrate.quad(lambda t: cf.ou_mean(a, b, r0, t), 0, T, epsabs=1e-14)[0]
        cov = lambda t, u: s * s / (2 * a) * (np.exp(-a * abs(t - u)) - np.exp(-a * (t + u)))
        v = integrate.dblquad(cov, 0, T, 0, T, epsabs=1e-14, epsrel=1e-12)[0]
        assert np.isclose(cf.vasicek_zc(a, b, s, r0, T), np.exp(-m + 0.5 * v), rtol=1e-9)


def test_cir_survival_matches_riccati_ode():
    k, th, nu, l0 = 0.5, 0.02, 0.1, 0.03

    def rhs(t, y):
        A, B = y
        return [k * th * B, 1.0 - k * B - 0.5 * nu * nu * B * B]

    for T in (1.0, 5.0, 10.0):
        sol = integrate.solve_ivp(rhs, (0, T), [0.0, 0.0], rtol=1e-12, atol=1e-14)
        A, B = sol.y[:, -1]
        assert np.isclose(cf.cir_survival(k, th, nu, l0, T), np.exp(-A - B * l0), rtol=1e-9)


# ------------------------------------------------------------------ simulation vs closed forms
@pytest.fixture(scope="module")
def plain_paths():
    w = wl.plain_fp64().with_(M=8192)
    return w, model.simulate_outer(w, np.arange(w.M))


def test_discount_factor_matches_vasicek_zc(plain_paths):
    w, o = plain_paths
    m = w.market
    n = w.grid.n_dates
    for i in (10, 25, 50):
        t = i * w.grid.horizon / n
        beta = np.exp(-o.I[i])
        zc = cf.vasicek_zc(m.a[0], m.b[0], m.sigma_r[0], m.r0[0], t)
        se = beta.std() / np.sqrt(beta.size)
        assert abs(beta.mean() - zc) < 5 * se + 2e-5


def test_short_rate_ou_moments(plain_paths):
    w, o = plain_paths
    m = w.market
    t = w.grid.horizon
    r = o.r[-1][:, 0]
    mean, var = cf.ou_mean(m.a[0], m.b[0], m.r0[0], t), cf.ou_var(m.a[0], m.sigma_r[0], t)
    assert abs(r.mean() - mean) < 5 * np.sqrt(var / r.size)
    assert abs(r.var() - var) < 5 * var * np.sqrt(2.0 / r.size)


def test_cir_survival_of_integrated_intensity(plain_paths):
    w, o = plain_paths
    m = w.market
    for i in (10, 50):
        t = i * w.grid.horizon / w.grid.n_dates
        s = np.exp(-o.Lam[i][:, 0])
        S = cf.cir_survival(m.kappa[0], m.theta[0], m.nu[0], m.lambda0[0], t)
        assert abs(s.mean() - S) < 5 * s.std() / np.sqrt(s.size) + 2e-4


@pytest.fixture(scope="module")
def two_ccy():
    w = two_ccy_workload()
    return w, model.simulate_outer(w, np.arange(w.M))


def test_fx_quanto_martingale(two_ccy):
    """E[beta_T chi_T] = chi_0 ZC^e_0(T) pins the quanto drift -rho sigma_r sigma_chi."""
    w, o = two_ccy
    m = w.market
    for i in (5, 10):
        t = i * w.grid.horizon / w.grid.n_dates
        y = np.exp(-o.I[i]) * np.exp(o.x[i][:, 0])
        target = m.fx0[0] * cf.vasicek_zc(m.a[1], m.b[1], m.sigma_r[1], m.r0[1], t)
        se = y.std() / np.sqrt(y.size)
        assert abs(y.mean() - target) < 5 * se + 1e-4 * target


def test_quanto_drift_as_printed_would_fail():
    """The drift printed without sigma^{r,e} is far off: the same test rejects it."""
    w = two_ccy_workload(M=4096)
    m = w.market
    rho = m.corr[1, 2]
    printed = rho * m.sigma_fx[0]
    ours = rho * m.sigma_r[1] * m.sigma_fx[0]
    # emulate the printed drift by shifting b^1 so that a (b' - r) - ours = a (b - r) - printed
    m2 = wl.Market(**{**m.__dict__, "b": np.array([m.b[0], m.b[1] - (printed - ours) / m.a[1]])})
    o = model.simulate_outer(w, np.arange(w.M), m2)
    t = w.grid.horizon
    y = np.exp(-o.I[-1]) * np.exp(o.x[-1][:, 0])
    target = m.fx0[0] * cf.vasicek_zc(m.a[1], m.b[1], m.sigma_r[1], m.r0[1], t)
    assert abs(y.mean() - target) > 10 * y.std() / np.sqrt(y.size)


def test_par_swap_has_zero_value_at_inception():
    w = two_ccy_workload()
    par = model.par_rates(w)
    for s in range(w.portfolio.n_swaps):
        e = w.portfolio.ccy[s]
        v = model.swap_value(w, s, 0, np.array([w.market.r0[e]]), None, par[s])
        assert abs(v[0]) < 1e-15


def test_swap_value_at_inception_closed_form():
    """P_0 = delta (par - Sigma) sum_k ZC_0(k delta) for any fixed rate Sigma."""
    w = two_ccy_workload()
    par = model.par_rates(w)
    m = w.market
    for s in range(w.portfolio.n_swaps):
        e = w.portfolio.ccy[s]
        Sig = par[s] + 0.0123
        ks = np.arange(1, w.portfolio.maturity[s] + 1)
        ann = sum(cf.vasicek_zc(m.a[e], m.b[e], m.sigma_r[e], m.r0[e], k) for k in ks)
        v = model.swap_value(w, s, 0, np.array([m.r0[e]]), None, Sig)
        assert np.isclose(v[0], (par[s] - Sig) * ann, rtol=1e-12, atol=1e-15)


def test_discounted_swap_is_martingale(two_ccy):
    """E[beta_i chi_i P_i] = chi_0 P_0 at reset and between-reset dates: pins the reset
    bookkeeping, the cum-coupon convention and the foreign measure change."""
    w, o = two_ccy
    fixed = model.fixed_rates(w)
    q = model.dates_per_reset(w)
    assert q == 1
    w5 = two_ccy_workload(n_dates=20, n_sub=20)   # two dates per reset period
    o5 = model.simulate_outer(w5, np.arange(w5.M))
    for ww, oo in ((w, o), (w5, o5)):
        q = model.dates_per_reset(ww)
        for s in range(ww.portfolio.n_swaps):
            e = ww.portfolio.ccy[s]
            fx0 = ww.market.fx0[e - 1] if e else 1.0
            P0 = model.swap_value(ww, s, 0, oo.r[0][:, e], None, fixed[s])[0]
            for i in range(1, int(ww.portfolio.maturity[s]) * q + 1):
                prev = (i - q) if i % q == 0 else (i // q) * q
                v = model.swap_value(ww, s, i, oo.r[i][:, e], oo.r[prev][:, e], fixed[s])
                fx = np.exp(oo.x[i][:, e - 1]) if e else 1.0
                y = np.exp(-oo.I[i]) * fx * v
                # cash flows paid at earlier reset dates are not in P_i: add them back
                paid = np.zeros_like(y)
                for k in range(q, i, q):
                    pk = (k - q)
                    cpn = 1.0 / model.zc(ww.market, e, oo.r[pk][:, e], ww.portfolio.delta) - 1.0 \
                        - ww.portfolio.delta * fixed[s]
                    fxk = np.exp(oo.x[k][:, e - 1]) if e else 1.0
                    paid += np.exp(-oo.I[k]) * fxk * cpn
                tot = y + paid
                se = tot.std() / np.sqrt(tot.size)
                assert abs(tot.mean() - fx0 * P0) < 5 * se + 2e-4, (s, i)


def test_features_layout():
    w = wl.small_multi(M=8)
    o = model.simulate_outer(w, np.arange(8))
    X = model.features(w, o)
    n_e, C = w.market.n_ccy, w.market.n_cpty
    assert X.shape == (w.grid.n_dates + 1, wl.n_features(w), 8)
    assert np.array_equal(X[3, 0], o.r[3][:, 0])
    assert np.array_equal(X[3, n_e], o.x[3][:, 0])
    assert np.array_equal(X[3, 2 * n_e - 1 + C], o.I[3])


def test_zero_volatility_reduces_to_geometric_recursion():
    """With sigma = nu = 0 the scheme is deterministic: r_k = b + (r0 - b)(1 - a dt)^k, and
    I, Lambda are trapezoid sums of that sequence, which have closed geometric-series forms."""
    w = two_ccy_workload(M=4, n_dates=5, n_sub=7)
    m = w.market
    m0 = wl.Market(**{**m.__dict__, "sigma_r": np.zeros(2), "sigma_fx": np.zeros(1),
                      "nu": np.zeros(1), "corr": np.eye(3)})
    o = model.simulate_outer(w, np.arange(4), m0)
    N = w.grid.n_dates * w.grid.n_sub
    dt = w.grid.horizon / N

    def geo_sum(q, k):      # sum_{j<k} q^j
        return (1.0 - q ** k) / (1.0 - q)

    def seq(a, b, x0, k):
        return b + (x0 - b) * (1.0 - a * dt) ** k

    def trap(a, b, x0, k):  # dt * sum_{j<k} (x_j + x_{j+1}) / 2
        q = 1.0 - a * dt
        return dt * (k * b + (x0 - b) * 0.5 * (geo_sum(q, k) + q * geo_sum(q, k)))

    k = N
    assert np.allclose(o.r[-1][:, 0], seq(m.a[0], m.b[0], m.r0[0], k), rtol=1e-13)
    assert np.allclose(o.I[-1], trap(m.a[0], m.b[0], m.r0[0], k), rtol=1e-12)
    assert np.allclose(o.g[-1][:, 0], seq(m.kappa[0], m.theta[0], m.lambda0[0], k), rtol=1e-13)
    assert np.allclose(o.Lam[-1][:, 0], trap(m.kappa[0], m.theta[0], m.lambda0[0], k), rtol=1e-12)
    # log FX: x_k = x_0 + dt sum_{j<k} (r0_j - r1_j); rho*sigma_r*sigma_fx = 0 here
    x_expect = np.log(m.fx0[0]) + dt * sum(
        seq(m.a[0], m.b[0], m.r0[0], j) - seq(m.a[1], m.b[1], m.r0[1], j) for j in range(k))
    assert np.allclose(o.x[-1][:, 0], x_expect, rtol=1e-12)
