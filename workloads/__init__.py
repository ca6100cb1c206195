"""Seeded synthetic inputs for the hierarchical-simulation CVA workloads.

This module only *draws* inputs: model parameters, a random correlation matrix and a
random swap book, as plain NumPy arrays.  It holds none of the method's arithmetic
(no zero-coupon prices, par rates, Cholesky factors, dynamics or payoffs), so that
both the FP64 oracle and the GPU library can consume the same inputs while sharing
no code.

The shapes follow the CVA case study (Section 4.3): n_e economies with Vasicek
short rates, n_e - 1 log-normal FX rates, C counterparties with CIR intensities,
a book of interest-rate swaps with random notional, currency, counterparty,
maturity and payer/receiver side, priced around par at inception.  Swap fixed
rates are given as a spread (in basis points) over the time-0 par rate; each side
turns the spread into a fixed rate with its own pricing code.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Dict, List, Optional

import numpy as np


@dataclass
class Market:
    """Model parameters (Appendix B, equations e:sde1 / e:sde2).

    Brownian ordering of the correlation matrix ``corr`` (size 2*n_e - 1):
    index e (0 <= e < n_e) drives r^e; index n_e + e - 1 (1 <= e < n_e) drives
    log chi^e.  CIR drivers are independent of the market block.
    """
    a: np.ndarray          # [n_e] Vasicek mean-reversion speed
    b: np.ndarray          # [n_e] Vasicek long-run level (under Q^e)
    sigma_r: np.ndarray    # [n_e] Vasicek volatility
    r0: np.ndarray         # [n_e] initial short rates
    sigma_fx: np.ndarray   # [n_e-1] FX log-volatility
    fx0: np.ndarray        # [n_e-1] initial FX rates (foreign -> domestic)
    corr: np.ndarray       # [2n_e-1, 2n_e-1] correlation of (B^r, B^chi)
    kappa: np.ndarray      # [C] CIR speed
    theta: np.ndarray      # [C] CIR long-run level
    nu: np.ndarray         # [C] CIR volatility
    lambda0: np.ndarray    # [C] initial intensity
    lgd: np.ndarray        # [C] loss given default

    @property
    def n_ccy(self) -> int:
        return int(self.a.shape[0])

    @property
    def n_cpty(self) -> int:
        return int(self.kappa.shape[0])


@dataclass
class Portfolio:
    """Swap book (Appendix B): annual resets, spot starting, maturities in whole years."""
    ccy: np.ndarray        # [S] int32 currency index
    cpty: np.ndarray       # [S] int32 counterparty index
    maturity: np.ndarray   # [S] int32 maturity in years (multiple of delta)
    notional: np.ndarray   # [S] float64, in the swap's currency
    spread_bp: np.ndarray  # [S] float64, fixed rate = par_0 + spread_bp * 1e-4
    payer: np.ndarray      # [S] int32, +1 bank pays fixed, -1 bank receives fixed
    delta: float = 1.0     # reset period in years

    @property
    def n_swaps(self) -> int:
        return int(self.ccy.shape[0])


@dataclass
class Grid:
    horizon: float   # years
    n_dates: int     # pricing dates n (date i at t_i = i * horizon / n)
    n_sub: int       # Euler sub-steps per pricing step


@dataclass
class MLPConfig:
    hidden: int = 2
    width: int = 32
    epochs: int = 200
    n_batches: Optional[int] = 32      # |B|; batch = M / |B|
    batch: Optional[int] = None        # or a fixed batch size
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    dtype: str = "fp32"


@dataclass
class Workload:
    name: str
    market: Market
    portfolio: Portfolio
    grid: Grid
    M: int
    n_b: int
    seed: int = 0
    features: str = "factors"          # "factors" or "factors_plus" (adds I_i, sum_c Lambda^c_i)
    mlp: MLPConfig = field(default_factory=MLPConfig)
    extra: Dict = field(default_factory=dict)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# --------------------------------------------------------------------------------------
# random correlation matrices: LKJ(eta) by the onion method
# (Lewandowski, Kurowicka & Joe, J. Multivariate Anal. 2009, Section 3.2)
# --------------------------------------------------------------------------------------
def lkj_corr(d: int, eta: float, rng: np.random.Generator) -> np.ndarray:
    if d == 1:
        return np.ones((1, 1))
    beta = eta + (d - 2) / 2.0
    r12 = 2.0 * rng.beta(beta, beta) - 1.0
    R = np.array([[1.0, r12], [r12, 1.0]])
    for k in range(2, d):
        beta -= 0.5
        y = rng.beta(k / 2.0, beta)
        u = rng.standard_normal(k)
        u /= np.linalg.norm(u)
        w = np.sqrt(y) * u
        A = np.linalg.cholesky(R)
        z = A @ w
        Rn = np.empty((k + 1, k + 1))
        Rn[:k, :k] = R
        Rn[:k, k] = z
        Rn[k, :k] = z
        Rn[k, k] = 1.0
        R = Rn
    return 0.5 * (R + R.T)


def random_book(rng: np.random.Generator, n_swaps: int, n_ccy: int, n_cpty: int,
                max_maturity: int = 10) -> Portfolio:
    ccy = rng.integers(0, n_ccy, size=n_swaps).astype(np.int32)
    cpty = rng.integers(0, n_cpty, size=n_swaps).astype(np.int32)
    maturity = rng.integers(1, max_maturity + 1, size=n_swaps).astype(np.int32)
    notional = rng.uniform(1e5, 1e6, size=n_swaps)
    spread_bp = rng.uniform(-50.0, 50.0, size=n_swaps)
    payer = np.where(rng.random(n_swaps) < 0.5, 1, -1).astype(np.int32)
    return Portfolio(ccy=ccy, cpty=cpty, maturity=maturity, notional=notional,
                     spread_bp=spread_bp, payer=payer)


# --------------------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------------------
def market_single(a=0.1, b=0.02, sigma=0.01, r0=0.02, kappa=0.5, theta=0.02, nu=0.1,
                  lambda0=0.02, lgd=0.6) -> Market:
    """One currency, one counterparty (the plain FP64 case)."""
    return Market(a=np.array([a]), b=np.array([b]), sigma_r=np.array([sigma]),
                  r0=np.array([r0]), sigma_fx=np.zeros(0), fx0=np.zeros(0),
                  corr=np.ones((1, 1)), kappa=np.array([kappa]), theta=np.array([theta]),
                  nu=np.array([nu]), lambda0=np.array([lambda0]), lgd=np.array([lgd]))


def market_multi(rng: np.random.Generator, n_ccy: int = 10, n_cpty: int = 8) -> Market:
    """n_ccy Vasicek rates, n_ccy-1 correlated GBM FX rates, n_cpty CIR intensities."""
    a = rng.uniform(0.05, 0.2, size=n_ccy)
    sigma_r = rng.uniform(0.005, 0.015, size=n_ccy)
    sigma_fx = rng.uniform(0.1, 0.3, size=n_ccy - 1)
    corr = lkj_corr(2 * n_ccy - 1, 2.0, rng)
    lambda0 = rng.uniform(0.005, 0.05, size=n_cpty)
    return Market(a=a, b=np.full(n_ccy, 0.02), sigma_r=sigma_r, r0=np.full(n_ccy, 0.02),
                  sigma_fx=sigma_fx, fx0=np.ones(n_ccy - 1), corr=corr,
                  kappa=np.full(n_cpty, 0.5), theta=np.full(n_cpty, 0.02),
                  nu=np.full(n_cpty, 0.1), lambda0=lambda0, lgd=np.full(n_cpty, 0.6))


def plain_fp64(seed: int = 0) -> Workload:
    """1 currency, 1 counterparty, 10 swaps, 50 dates over 10y, M=1024, n_b=16."""
    rng = np.random.default_rng(seed)
    book = random_book(rng, 10, 1, 1)
    return Workload(name="plain_fp64_1ccy_1cpty_10swaps_M1024_nb16", market=market_single(),
                    portfolio=book, grid=Grid(10.0, 50, 25), M=1024, n_b=16, seed=seed,
                    mlp=MLPConfig(hidden=2, width=32, epochs=200, n_batches=32))


def cva_at_scale(seed: int = 0, M: int = 1 << 17, n_b: int = 128) -> Workload:
    """10 currencies, 9 FX, 8 counterparties, 500 swaps, 100 dates, M=2^17, n_b=128."""
    rng = np.random.default_rng(seed)
    mkt = market_multi(rng, 10, 8)
    book = random_book(rng, 500, 10, 8)
    return Workload(name=f"cva_10ccy_8cpty_500swaps_100dates_M{M}_nb{n_b}", market=mkt,
                    portfolio=book, grid=Grid(10.0, 100, 25), M=M, n_b=n_b, seed=seed,
                    features="factors_plus",
                    mlp=MLPConfig(hidden=3, width=128, epochs=50, n_batches=None,
                                  batch=8192, dtype="bf16"))


OVERSIM_LEVELS = (1, 8, 64, 512, 1024)


def oversim_sweep(M: int, seed: int = 0, block_paths: int = 64,
                  levels=OVERSIM_LEVELS) -> Workload:
    """Plain-case market; block b of `block_paths` outer paths gets n_b = levels[b % 5]."""
    w = plain_fp64(seed)
    nblk = (M + block_paths - 1) // block_paths
    nb_blocks = np.array([levels[b % len(levels)] for b in range(nblk)], dtype=np.int32)
    return w.with_(name=f"oversim_sweep_M{M}", M=M, n_b=int(max(levels)),
                   extra={"block_paths": block_paths, "n_b_per_block": nb_blocks})


def precision_form(seed: int = 0, M: int = 1 << 17) -> Workload:
    w = cva_at_scale(seed, M=M, n_b=128)
    return w.with_(name=f"bf16_batched_fit_100dates_M{M}")


def differentiation_form(seed: int = 0, M: int = 1 << 16) -> Workload:
    w = cva_at_scale(seed, M=M, n_b=64)
    return w.with_(name=f"adjoint_90params_M{M}_nb64", extra={"ckpt_every": 10})


def tiny(seed: int = 0, n_ccy: int = 2, n_cpty: int = 2, n_swaps: int = 3,
         n_dates: int = 4, n_sub: int = 2, horizon: float = 2.0, M: int = 2,
         n_b: int = 3) -> Workload:
    """Brute-force sized case: everything enumerable by hand."""
    rng = np.random.default_rng(1000 + seed)
    mkt = market_multi(rng, n_ccy, n_cpty) if n_ccy > 1 else market_single()
    if n_ccy == 1 and n_cpty > 1:
        mkt = replace(mkt, kappa=np.full(n_cpty, 0.5), theta=np.full(n_cpty, 0.02),
                      nu=np.full(n_cpty, 0.1), lambda0=rng.uniform(0.01, 0.05, n_cpty),
                      lgd=np.full(n_cpty, 0.6))
    book = random_book(rng, n_swaps, n_ccy, n_cpty, max_maturity=int(horizon))
    return Workload(name="tiny", market=mkt, portfolio=book,
                    grid=Grid(horizon, n_dates, n_sub), M=M, n_b=n_b, seed=seed,
                    mlp=MLPConfig(hidden=1, width=32, epochs=4, n_batches=2))


def small_multi(seed: int = 0, M: int = 256, n_b: int = 8, n_ccy: int = 3, n_cpty: int = 3,
                n_swaps: int = 40, n_dates: int = 20, n_sub: int = 5,
                horizon: float = 10.0) -> Workload:
    """A few-currency case that the oracle finishes in seconds; spans several tiles."""
    rng = np.random.default_rng(2000 + seed)
    mkt = market_multi(rng, n_ccy, n_cpty)
    book = random_book(rng, n_swaps, n_ccy, n_cpty, max_maturity=int(horizon))
    return Workload(name=f"small_{n_ccy}ccy_{n_cpty}cpty_M{M}", market=mkt, portfolio=book,
                    grid=Grid(horizon, n_dates, n_sub), M=M, n_b=n_b, seed=seed,
                    features="factors_plus",
                    mlp=MLPConfig(hidden=2, width=32, epochs=6, n_batches=4))


def get(name: str, **kw) -> Workload:
    table = {"plain_fp64": plain_fp64, "cva_at_scale": cva_at_scale,
             "oversim_sweep": oversim_sweep, "precision_form": precision_form,
             "differentiation_form": differentiation_form, "tiny": tiny,
             "small_multi": small_multi}
    return table[name](**kw)


def n_features(w: Workload) -> int:
    m = w.market
    d = m.n_ccy + (m.n_ccy - 1) + m.n_cpty
    return d + 2 if w.features == "factors_plus" else d


__all__ = ["Market", "Portfolio", "Grid", "MLPConfig", "Workload", "lkj_corr", "random_book",
           "market_single", "market_multi", "plain_fp64", "cva_at_scale", "oversim_sweep",
           "precision_form", "differentiation_form", "tiny", "small_multi", "get",
           "n_features", "OVERSIM_LEVELS"]
