"""Outer market simulation and swap pricing (FP64 oracle).

Follows Appendix B (equations e:sde1, e:sde2, the Girsanov change to Q^0 for
foreign short rates, the default rule e:tau and the three-case swap price) and
Remark rem:finecoarse of Section 4.1 (Euler stepping on a fine grid, numerical
integration of r^0 and of the intensities on that grid, storage at pricing dates
only).

Readings taken where the paper is silent or garbled:
  * Euler-Maruyama with every drift and diffusion coefficient taken at the old state.
  * Foreign short rates under Q^0: the printed drift correction omits sigma^{r,e};
    the Girsanov step it comes from gives  -rho^e sigma^{r,e} sigma^{chi,e}.
  * CIR negativity: full truncation, gamma^+ in drift and diffusion.
  * Integrals I = int r^0 and Lambda^c = int gamma^{c,+}: trapezoid rule on the
    fine grid, accumulated in FP64.
  * Reset dates are recognised by integer date arithmetic: with q = n delta / T
    pricing dates per reset period, date i is a reset date iff i mod q == 0.
  * At a reset date t > 0 the swap value is cum-coupon (the second printed case).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import philox
from .closed_forms import vasicek_zc


@dataclass
class OuterPaths:
    r: np.ndarray      # [n+1, P, n_e] short rates at pricing dates
    x: np.ndarray      # [n+1, P, n_e-1] log FX rates
    g: np.ndarray      # [n+1, P, C] intensities
    I: np.ndarray      # [n+1, P] int_0^{t_i} r^0  (beta_i = exp(-I_i))
    Lam: np.ndarray    # [n+1, P, C] int_0^{t_i} gamma^{c,+}


def dims(w):
    n_e, C = w.market.n_ccy, w.market.n_cpty
    d_w = 2 * n_e - 1
    return n_e, C, d_w, d_w + C


def dates_per_reset(w) -> int:
    g, d = w.grid, w.portfolio.delta
    q = g.n_dates * d / g.horizon
    if abs(q - round(q)) > 1e-12 or round(q) < 1:
        raise ValueError("reset period must be a whole number of pricing steps")
    return int(round(q))


def simulate_outer(w, paths, market=None, branch=None, branch_date: int = 0) -> OuterPaths:
    """Euler scheme of Appendix B on the fine grid; values stored at the pricing dates.

    With ``branch`` (one continuation index per entry of ``paths``), the sub-steps of
    dates after ``branch_date`` draw the branch normals of that continuation: up to
    t_{branch_date} the path is the outer path itself, afterwards a conditionally
    independent copy of its future (the re-simulation of Section 3.3's twin Monte
    Carlo and of the nested Monte Carlo benchmark of Section 4.3).
    """
    m = w.market if market is None else market
    n_e, C, d_w, n_z = dims(w)
    n, n_sub = w.grid.n_dates, w.grid.n_sub
    dt = w.grid.horizon / (n * n_sub)
    sq = np.sqrt(dt)
    L = np.linalg.cholesky(m.corr)
    rho = np.array([m.corr[e, n_e + e - 1] for e in range(1, n_e)])
    paths = np.asarray(paths, dtype=np.int64)
    P = paths.shape[0]

    r = np.tile(np.asarray(m.r0, dtype=np.float64), (P, 1))
    x = np.tile(np.log(np.asarray(m.fx0, dtype=np.float64)), (P, 1))
    g = np.tile(np.asarray(m.lambda0, dtype=np.float64), (P, 1))
    I = np.zeros(P)
    Lam = np.zeros((P, C))

    out = OuterPaths(r=np.empty((n + 1, P, n_e)), x=np.empty((n + 1, P, n_e - 1)),
                     g=np.empty((n + 1, P, C)), I=np.empty((n + 1, P)),
                     Lam=np.empty((n + 1, P, C)))

    def store(i):
        out.r[i], out.x[i], out.g[i], out.I[i], out.Lam[i] = r, x, g, I, Lam

    store(0)
    for i in range(n):
        for j in range(n_sub):
            s = i * n_sub + j
            if branch is not None and i >= branch_date:
                z = philox.outer_normals(w.seed, paths, s, n_z, branch=branch)
            else:
                z = philox.outer_normals(w.seed, paths, s, n_z)
            Wc = z[:, :d_w] @ L.T                        # correlated market increments
            r_old, g_old = r.copy(), np.maximum(g, 0.0)
            # domestic Vasicek under Q^0
            r[:, 0] = r_old[:, 0] + m.a[0] * (m.b[0] - r_old[:, 0]) * dt \
                + m.sigma_r[0] * sq * Wc[:, 0]
            for e in range(1, n_e):
                quanto = rho[e - 1] * m.sigma_r[e] * m.sigma_fx[e - 1]
                r[:, e] = r_old[:, e] + (m.a[e] * (m.b[e] - r_old[:, e]) - quanto) * dt \
                    + m.sigma_r[e] * sq * Wc[:, e]
                x[:, e - 1] = x[:, e - 1] + (r_old[:, 0] - r_old[:, e]
                                             - 0.5 * m.sigma_fx[e - 1] ** 2) * dt \
                    + m.sigma_fx[e - 1] * sq * Wc[:, n_e + e - 1]
            for c in range(C):
                g[:, c] = g[:, c] + m.kappa[c] * (m.theta[c] - g_old[:, c]) * dt \
                    + m.nu[c] * np.sqrt(g_old[:, c]) * sq * z[:, d_w + c]
            I = I + 0.5 * (r_old[:, 0] + r[:, 0]) * dt
            Lam = Lam + 0.5 * (g_old + np.maximum(g, 0.0)) * dt
        store(i + 1)
    return out


# ---------------------------------------------------------------------------------------
# pricing (Appendix B, three-case swap formula)
# ---------------------------------------------------------------------------------------
def zc(m, e, r, tau):
    return vasicek_zc(m.a[e], m.b[e], m.sigma_r[e], r, tau)


def par_rates(w, market=None) -> np.ndarray:
    """Time-0 par rate of every swap: the fixed rate for which the t=0 case is zero."""
    m = w.market if market is None else market
    pf, d = w.portfolio, w.portfolio.delta
    out = np.empty(pf.n_swaps)
    for s in range(pf.n_swaps):
        e, tbar = pf.ccy[s], float(pf.maturity[s])
        k = np.arange(1, int(round(tbar / d)) + 1)
        ann = d * np.sum(zc(m, e, m.r0[e], k * d))
        out[s] = (1.0 - zc(m, e, m.r0[e], tbar)) / ann
    return out


def fixed_rates(w, market=None) -> np.ndarray:
    return par_rates(w, market) + 1e-4 * np.asarray(w.portfolio.spread_bp)


def swap_value(w, s, i, r_now, r_prev_reset, Sigma, market=None):
    """P^sw_{t_i} of swap s in its own currency, given r^e at t_i and at the last reset.

    r_prev_reset is r^e at the reset date strictly before t_i when t_i is a reset
    date, and at the reset date t_- <= t_i otherwise.
    """
    m = w.market if market is None else market
    pf, d = w.portfolio, w.portfolio.delta
    q = dates_per_reset(w)
    h = w.grid.horizon / w.grid.n_dates                 # years per pricing step
    e = pf.ccy[s]
    mat_idx = int(pf.maturity[s]) * q                   # t-bar as a date index (delta = q steps)
    if i > mat_idx:
        return np.zeros_like(r_now)
    t = i * h
    tbar = mat_idx * h
    later = [k for k in range(q, mat_idx + 1, q) if k > i]   # reset dates t' > t
    ann = sum(zc(m, e, r_now, kk * h - t) for kk in later) if later else 0.0
    if i == 0:
        return 1.0 - zc(m, e, r_now, tbar) - d * Sigma * ann
    if i % q == 0:
        coupon = 1.0 / zc(m, e, r_prev_reset, d)
        return coupon - zc(m, e, r_now, tbar - t) - d * Sigma * (1.0 + ann)
    t_plus = (i // q) * q + q
    t_minus = (i // q) * q
    ratio = zc(m, e, r_now, t_plus * h - t) / zc(m, e, r_prev_reset, (t_plus - t_minus) * h)
    return ratio - zc(m, e, r_now, tbar - t) - d * Sigma * ann


def mtm(w, outer: OuterPaths, fixed=None, market=None) -> np.ndarray:
    """MtM^c_i in the reference currency: [n+1, P, C]."""
    m = w.market if market is None else market
    pf = w.portfolio
    n, C = w.grid.n_dates, m.n_cpty
    q = dates_per_reset(w)
    fixed = fixed_rates(w, m) if fixed is None else fixed
    P = outer.I.shape[1]
    out = np.zeros((n + 1, P, C))
    for i in range(n + 1):
        prev = (i - q) if (i % q == 0 and i > 0) else (i // q) * q
        for s in range(pf.n_swaps):
            e = pf.ccy[s]
            v = swap_value(w, s, i, outer.r[i][:, e], outer.r[prev][:, e], fixed[s], m)
            fx = np.exp(outer.x[i][:, e - 1]) if e > 0 else 1.0
            out[i][:, pf.cpty[s]] += pf.payer[s] * pf.notional[s] * fx * v
    return out


def exposure(w, outer: OuterPaths, mtm_c: np.ndarray, market=None) -> np.ndarray:
    """D^c_i = LGD_c beta_i (MtM^c_i)^+ : [n+1, P, C]."""
    m = w.market if market is None else market
    beta = np.exp(-outer.I)
    return m.lgd[None, None, :] * beta[:, :, None] * np.maximum(mtm_c, 0.0)


def features(w, outer: OuterPaths) -> np.ndarray:
    """Regression inputs at each date: [n+1, d, P].

    Market factors (r^0..r^{n_e-1}, log chi^1..log chi^{n_e-1}, gamma^1..gamma^C),
    the 27 diffusive factors of Section 4.3 in the ten-currency case, optionally
    followed by I_i = -log beta_i and sum_c Lambda^c_i.
    """
    f = [outer.r, outer.x, outer.g]
    if w.features == "factors_plus":
        f += [outer.I[:, :, None], outer.Lam.sum(axis=2, keepdims=True)]
    X = np.concatenate(f, axis=2)            # [n+1, P, d]
    return np.ascontiguousarray(np.transpose(X, (0, 2, 1)))
