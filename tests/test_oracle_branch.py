"""Pins of the branched re-simulation oracle (nested / twin Monte Carlo, Sections 3.3 and 4.3).

  * the continuation is the outer path itself up to the branching date, bit for bit, and a
    different path (per branch) after it;
  * with deterministic rates, the mean over continuations of the intensity-form sample equals
    the CIR closed form of the conditional survival increments (a textbook formula that
    shares nothing with the simulation);
  * the twin estimator is unbiased for E[(phi - CVA)^2] on samples of known conditional mean,
    where the nested estimator is biased by E[Var]/B, and reduces to e:val1 for B = 2;
  * tower property: the average of the nested estimates equals the average intensity target
    of independent outer paths.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import branch, closed_forms, model, pipeline


def test_prefix_is_the_outer_path_and_branches_differ_after():
    w = wl.small_multi(M=16, n_dates=10, n_sub=3)
    paths = np.arange(5, 13)
    date = 4
    ref = model.simulate_outer(w, paths)
    B = 3
    lane_path = np.tile(paths, B)
    lane_branch = np.repeat(np.arange(B), paths.size)
    br = model.simulate_outer(w, lane_path, branch=lane_branch, branch_date=date)
    for name in ("r", "x", "g", "I", "Lam"):
        a = getattr(ref, name)
        b = getattr(br, name)
        for bb in range(B):
            sl = slice(bb * paths.size, (bb + 1) * paths.size)
            assert np.array_equal(a[:date + 1], b[:date + 1, sl]), name
            assert not np.any(a[date + 1:] == b[date + 1:, sl]) or name == "x" and a.size == 0
    # distinct continuations of the same path differ from each other
    r1 = br.r[date + 1:, :paths.size]
    r2 = br.r[date + 1:, paths.size:2 * paths.size]
    assert not np.any(r1 == r2)


def test_last_date_has_nothing_left():
    w = wl.tiny(M=3)
    xi = branch.branch_targets(w, np.arange(3), w.grid.n_dates, 2)
    assert np.all(xi == 0.0)


def test_deterministic_rates_match_cir_closed_form():
    m = wl.market_single(sigma=0.0)
    w = wl.plain_fp64().with_(market=m, M=1)
    date, B = 20, 16384
    xi = branch.branch_targets(w, np.array([0]), date, B)[:, 0]
    # the state at the branching date and the (deterministic) exposures
    o = model.simulate_outer(w, np.array([0]))
    D = model.exposure(w, o, model.mtm(w, o))[:, 0, 0]
    h = w.grid.horizon / w.grid.n_dates
    g_i, Lam_i, I_i = o.g[date, 0, 0], o.Lam[date, 0, 0], o.I[date, 0]
    S = lambda tau: closed_forms.cir_survival(m.kappa[0], m.theta[0], m.nu[0], g_i, tau)
    exact = sum(np.exp(I_i) * D[j] * np.exp(-Lam_i) * (S((j - 1 - date) * h) - S((j - date) * h))
                for j in range(date + 1, w.grid.n_dates + 1))
    err = abs(xi.mean() - exact)
    se = xi.std(ddof=1) / np.sqrt(B)
    print(f"  nested mean {xi.mean():.6e}, CIR closed form {exact:.6e}, "
          f"diff {err / se:.2f} standard errors")
    # Monte Carlo error plus the Euler / trapezoid bias of the fine grid (dt = 0.008)
    assert err <= 4.0 * se + 2e-3 * exact


def test_twin_estimator_on_samples_of_known_mean():
    rng = np.random.default_rng(7)
    P, B = 200_000, 2
    cva = rng.lognormal(-3.0, 0.5, P)
    delta = 0.1 * cva * rng.standard_normal(P)
    phi = cva + delta
    noise_sd = 0.8 * cva
    xi = cva[None, :] + noise_sd[None, :] * rng.standard_normal((B, P))
    st = branch.twin_errors(phi, xi)
    true_mse = float(np.mean(delta ** 2))
    # e:val1 for two copies, term by term
    val1 = np.mean(phi ** 2 - (xi[0] + xi[1]) * phi + xi[0] * xi[1])
    assert st["mse_twin"] == pytest.approx(val1, rel=1e-12)
    # unbiased: within a few standard errors of the true L^2 error
    terms = phi ** 2 - 2 * phi * xi.mean(0) + xi[0] * xi[1]
    se = terms.std() / np.sqrt(P)
    assert abs(st["mse_twin"] - true_mse) < 4 * se
    # the nested estimator carries the inner variance / B
    bias = float(np.mean(noise_sd ** 2)) / B
    assert st["mse_nested"] == pytest.approx(true_mse + bias, rel=0.02)
    assert st["cva_sq"] == pytest.approx(float(np.mean(cva ** 2)), rel=0.02)
    assert st["cva_mean"] == pytest.approx(float(np.mean(cva)), rel=0.01)
    # more continuations: the U-statistic stays unbiased for E[CVA^2]
    xi8 = cva[None, :] + noise_sd[None, :] * rng.standard_normal((8, P))
    st8 = branch.twin_errors(phi, xi8)
    assert st8["cva_sq"] == pytest.approx(float(np.mean(cva ** 2)), rel=0.01)
    assert st8["cva_sq_nested"] - st8["cva_sq"] == pytest.approx(
        float(np.mean(xi8.var(axis=0, ddof=1))) / 8, rel=1e-9)


def test_nested_estimates_average_to_the_intensity_targets():
    w = wl.small_multi(M=4096, n_dates=10, n_sub=3)
    date = 4
    ref = pipeline.simulate(w, with_moments=True, n_b=1)
    P = 1024
    xi = branch.branch_targets(w, np.arange(w.M, w.M + P), date, 4)   # paths not in ref
    a = xi.mean()
    b = ref["mu"][date].mean()
    se = np.sqrt(xi.mean(0).var(ddof=1) / P + ref["mu"][date].var(ddof=1) / w.M)
    print(f"  nested {a:.5e} vs outer {b:.5e} ({abs(a - b) / se:.2f} se)")
    assert abs(a - b) < 4 * se
