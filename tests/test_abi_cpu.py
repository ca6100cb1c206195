"""The C-ABI library loads, exports every declared symbol, and validates arguments on the
host before any launch (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as wl
from oracle import model

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hsim.h")


@pytest.fixture(scope="module")
def hs():
    from paper_2211_17005_amd import hsim
    if not os.path.exists(hsim.LIB_PATH):
        pytest.skip("libhsim.so not built")
    return hsim


def declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|size_t|const char\*)\s+(\w+)\(", txt, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("hsim_outer_paths", "hsim_inner_defaults", "hsim_targets_cva",
                     "hsim_inner_defaults_cva", "hsim_philox_fill", "cva_regress_fit",
                     "cva_regress_predict"):
        assert required in names, required


def test_library_exports_every_declared_symbol(hs):
    L = ctypes.CDLL(hs.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name


def test_abi_version(hs):
    assert hs.abi_version() == 3


def test_par_rates_match_oracle(hs):
    for w in (wl.plain_fp64(), wl.cva_at_scale(M=64), wl.small_multi()):
        assert np.allclose(hs.par_rates(w.market, w.portfolio), model.par_rates(w), rtol=1e-13,
                           atol=0)


def test_n_features(hs):
    w = wl.cva_at_scale(M=64)
    assert hs.n_features(w.market, hs.FEAT_FACTORS) == 27
    assert hs.n_features(w.market, hs.FEAT_FACTORS_PLUS) == 29
    assert hs.n_features(wl.plain_fp64().market, hs.FEAT_FACTORS) == 2


@pytest.fixture
def cpu_only():
    """These calls pass placeholder pointers that validation must reject; never on a GPU."""
    from conftest import gpu_available
    if gpu_available():
        pytest.skip("placeholder-pointer validation tests run on CPU only")


def call_outer(hs, w, market=None, book=None, grid=None, M=64, precision=1, fixed=None):
    m = w.market if market is None else market
    km = hs.market_struct(m)
    b = w.portfolio if book is None else book
    fixed = np.zeros(len(b.ccy)) if fixed is None else fixed
    kp = hs.portfolio_struct(b, fixed)
    g = hs.grid_struct(w.grid if grid is None else grid)
    dummy = ctypes.c_void_p(16)      # never dereferenced: validation fails first
    rc = hs.lib().hsim_outer_paths(ctypes.byref(km.struct), ctypes.byref(kp.struct),
                                   ctypes.byref(g), 0, 0, M, precision, 0, None, dummy, dummy,
                                   dummy, None, None)
    return rc, hs.lib().hsim_last_error().decode()


def test_rejects_bad_arguments_before_launch(hs, cpu_only):
    w = wl.small_multi()
    m = w.market
    # M <= 0
    rc, msg = call_outer(hs, w, M=0)
    assert rc == -1 and "M" in msg
    # correlation not positive definite
    c = m.corr.copy()
    c[0, 1] = c[1, 0] = 1.5
    rc, msg = call_outer(hs, w, market=wl.Market(**{**m.__dict__, "corr": c}))
    assert rc == -1 and "positive definite" in msg
    # non-unit diagonal
    bad2 = wl.Market(**{**m.__dict__, "corr": 2.0 * m.corr})
    rc, msg = call_outer(hs, w, market=bad2)
    assert rc == -1 and "diagonal" in msg
    # a <= 0
    bad3 = wl.Market(**{**m.__dict__, "a": -m.a})
    rc, _ = call_outer(hs, w, market=bad3)
    assert rc == -1
    # unsupported shape
    w4 = wl.small_multi(n_ccy=4, n_cpty=4)
    rc, msg = call_outer(hs, w4)
    assert rc == -5
    # maturity beyond the horizon
    b = wl.Portfolio(**{**w.portfolio.__dict__, "maturity": w.portfolio.maturity + 20})
    rc, msg = call_outer(hs, w, book=b)
    assert rc == -1 and "horizon" in msg
    # reset period not a whole number of steps
    rc, msg = call_outer(hs, w, grid=wl.Grid(10.0, 15, 2))
    assert rc == -1 and "whole number" in msg
    # payer must be +-1
    b = wl.Portfolio(**{**w.portfolio.__dict__, "payer": np.zeros(w.portfolio.n_swaps, np.int32)})
    rc, _ = call_outer(hs, w, book=b)
    assert rc == -1
    # unknown precision
    rc, _ = call_outer(hs, w, precision=7)
    assert rc == -1


def test_fused_rejects_small_workspace(hs, cpu_only):
    w = wl.small_multi()
    km = hs.market_struct(w.market)
    kp = hs.portfolio_struct(w.portfolio, np.zeros(w.portfolio.n_swaps))
    g = hs.grid_struct(w.grid)
    need = hs.lib().hsim_workspace_bytes(hs.OP_FUSED, ctypes.byref(km.struct), ctypes.byref(g),
                                         w.M, 1)
    assert need > 0
    dummy = ctypes.c_void_p(256)
    rc = hs.lib().hsim_inner_defaults_cva(ctypes.byref(km.struct), ctypes.byref(kp.struct),
                                          ctypes.byref(g), 0, 0, w.M, 8, None, 64, 1, 0, None,
                                          dummy, dummy, dummy, need - 1, None)
    assert rc == -3


def test_one_launch_rejects_bad_arguments(hs, cpu_only):
    """hsim_fused: workspace too small, FP32_PLAIN (not a form of the one-launch kernel), and a
    date x counterparty table beyond its LDS are refused before any launch; the inner stage
    refuses more dates than its LDS tile holds."""
    w = wl.small_multi()
    km = hs.market_struct(w.market)
    kp = hs.portfolio_struct(w.portfolio, np.zeros(w.portfolio.n_swaps))
    g = hs.grid_struct(w.grid)
    need = hs.lib().hsim_workspace_bytes(hs.OP_FUSED_LAUNCH, ctypes.byref(km.struct), ctypes.byref(g), w.M, 1)
    assert need > 0
    dummy = ctypes.c_void_p(256)
    call = lambda g_, prec, ws: hs.lib().hsim_fused(ctypes.byref(km.struct), ctypes.byref(kp.struct),
                                                    ctypes.byref(g_), 0, 0, w.M, 8, None, 64, prec, 0, None,
                                                    dummy, dummy, dummy, ws, None)
    assert call(g, 1, need - 1) == -3
    assert call(g, hs.HSIM_FP32_PLAIN, need) == -1
    keep = lambda n_keep, ptr: hs.lib().hsim_fused_keep(ctypes.byref(km.struct), ctypes.byref(kp.struct),
                                                       ctypes.byref(g), 0, 0, w.M, 8, None, 64, 1, 0, None,
                                                       dummy, dummy, n_keep, ptr, ptr, ptr, dummy, need, None)
    assert keep(w.M + 1, dummy) == -1 and b"n_keep" in hs.lib().hsim_last_error()
    assert keep(-1, dummy) == -1
    assert keep(5, None) == -1 and b"NULL" in hs.lib().hsim_last_error()
    big = hs.grid_struct(wl.Grid(8.0, 512, 5))        # 513 dates x 16 counterparties: 104 KiB of LDS
    m16 = hs.market_struct(wl.small_multi(n_cpty=16).market)
    need16 = hs.lib().hsim_workspace_bytes(hs.OP_FUSED_LAUNCH, ctypes.byref(m16.struct), ctypes.byref(big), 64, 1)
    rc = hs.lib().hsim_fused(ctypes.byref(m16.struct), ctypes.byref(kp.struct), ctypes.byref(big), 0, 0, 64, 8,
                             None, 64, 1, 0, None, dummy, dummy, dummy, need16, None)
    assert rc == -2 and b"LDS" in hs.lib().hsim_last_error()
    assert hs.lib().hsim_inner_defaults(ctypes.byref(big), 1, 0, 0, 64, 8, None, 64, dummy, dummy,
                                        None, 0, None) == -2


def test_inner_rejects_bad_nb(hs, cpu_only):
    g = hs.grid_struct(wl.Grid(10.0, 50, 25))
    dummy = ctypes.c_void_p(256)
    assert hs.lib().hsim_inner_defaults(ctypes.byref(g), 1, 0, 0, 64, 0, None, 64, dummy, dummy,
                                        None, 0, None) == -2
    assert hs.lib().hsim_inner_defaults(ctypes.byref(g), 1, 0, 0, 64, 1, dummy, 48, dummy, dummy,
                                        None, 0, None) == -1
    # uneven n_b runs longest-first from a work list kept in the workspace
    need = hs.lib().hsim_workspace_bytes(hs.OP_INNER, None, ctypes.byref(g), 64, hs.HSIM_FP32)
    assert need > 0
    assert hs.lib().hsim_inner_defaults(ctypes.byref(g), 1, 0, 0, 64, 0, dummy, 64, dummy, dummy,
                                        None, 0, None) == -3
    assert hs.lib().hsim_inner_defaults(ctypes.byref(g), 1, 0, 0, 64, 0, dummy, 64, dummy, dummy,
                                        dummy, need - 1, None) == -3


def test_intensity_targets_reject_bad_arguments(hs, cpu_only):
    g = hs.grid_struct(wl.Grid(10.0, 50, 25))
    dummy = ctypes.c_void_p(256)
    need = hs.lib().hsim_workspace_bytes(hs.OP_TARGETS, None, ctypes.byref(g), 64, hs.HSIM_FP32)
    f = hs.lib().hsim_targets_intensity
    assert f(ctypes.byref(g), 0, 64, 1, dummy, dummy, dummy, dummy, dummy, dummy, need, None) == -2
    assert f(ctypes.byref(g), 1, 0, 1, dummy, dummy, dummy, dummy, dummy, dummy, need, None) == -1
    assert f(ctypes.byref(g), 1, 64, 1, dummy, None, dummy, dummy, dummy, dummy, need, None) == -1
    assert f(ctypes.byref(g), 1, 64, 1, dummy, dummy, dummy, dummy, dummy, dummy, need - 1,
             None) == -3


def test_branch_entry_points_reject_bad_arguments(hs, cpu_only):
    w = wl.small_multi()
    km = hs.market_struct(w.market)
    kp = hs.portfolio_struct(w.portfolio, np.zeros(w.portfolio.n_swaps))
    g = hs.grid_struct(w.grid)
    dummy = ctypes.c_void_p(256)
    f = hs.lib().hsim_branch_cva
    args = (ctypes.byref(km.struct), ctypes.byref(kp.struct), ctypes.byref(g), 0, 0)
    assert f(*args, 64, -1, 2, 1, dummy, None) == -1                     # date < 0
    assert f(*args, 64, w.grid.n_dates + 1, 2, 1, dummy, None) == -1     # date > n
    assert f(*args, 64, 3, 0, 1, dummy, None) == -2                      # no continuation
    assert f(*args, 1 << 20, 3, 1 << 12, 1, dummy, None) == -2           # M * B > 2^31
    assert f(*args, 64, 3, 2, 1, None, None) == -1                       # no output
    e = hs.lib().hsim_branch_errors
    need = hs.lib().hsim_workspace_bytes(hs.OP_BRANCH, None, None, 1000, 1)
    assert need >= 6 * 4 * 8
    assert e(1000, 1, 1, None, dummy, dummy, dummy, need, None) == -2   # B < 2
    assert e(1000, 2, 1, None, dummy, dummy, dummy, need - 1, None) == -3
    assert e(0, 2, 1, None, dummy, dummy, dummy, need, None) == -1


def test_sample_rows_reject_bad_arguments(hs, cpu_only):
    g = hs.grid_struct(wl.Grid(10.0, 50, 25))
    dummy = ctypes.c_void_p(256)
    f = hs.lib().hsim_sample_rows
    ok = (dummy, dummy, dummy, dummy, dummy, dummy, None)
    assert f(ctypes.byref(g), 0, 2, 0, 0, 64, 4, 1, *ok) == -2            # n_cpty
    assert f(ctypes.byref(g), 1, 2, 0, 0, 64, 0, 1, *ok) == -2            # n_b
    assert f(ctypes.byref(g), 1, 2, 0, 0, 1 << 28, 16, 1, *ok) == -2      # M n_b > 2^31
    assert f(ctypes.byref(g), 1, 2, 0, 0, 64, 4, 1, None, dummy, dummy, dummy, dummy, dummy,
             None) == -1                                                  # features


def test_oversim_chooser_matches_oracle(hs):
    """hsim_oversim_choose / hsim_oversim_cost_ratio (host arithmetic of Section 3.3) against the
    oracle's Proposition p:heurisN, Heuristic heur:MN and l:ratio on seeded pilot moments, with
    dates whose R or Q rule N* out (no loss after the last maturity, a negative R)."""
    from oracle import oversim as oos
    rng = np.random.default_rng(5)
    A = rng.gamma(2.0, 1.0, (12, 4000)) * rng.random((12, 1))          # per outer path
    g1 = A + rng.gamma(1.5, 1.0, (12, 4000))                          # two continuations
    g2 = A + rng.gamma(1.5, 1.0, (12, 4000))
    g1[10:], g2[10:] = 0.0, 0.0                          # dates after the last maturity
    mom = oos.moments(g1, g2)
    mom[3, 2] = mom[3, 0] ** 2 - 1e-3                    # a date with R < 0
    P = oos.cost_ratio(0.31, 0.95, 1.0, 256.0)
    assert np.isclose(hs.oversim_cost_ratio(0.31, 0.95, 1.0, 256.0), P, rtol=1e-15)
    out = hs.oversim_choose(mom, P, 1e9)
    R, Q = oos.r_and_q(mom)
    ok = (R > 0) & (Q >= 0)
    assert out["defined"] == ok.sum() == 9
    assert np.allclose(out["R"], R, rtol=1e-15, atol=0) and np.allclose(out["Q"], Q, rtol=1e-15, atol=0)
    assert np.array_equal(np.isfinite(out["N_dates"]), ok)
    Ns = oos.optimal_n(Q[ok], R[ok], P)
    assert np.allclose(out["N_dates"][ok], Ns, rtol=1e-14)
    N, M = oos.heuristic(Ns, P, 1e9)
    assert np.isclose(out["N"], N, rtol=1e-14) and np.isclose(out["M"], M, rtol=1e-14)
    small = hs.oversim_choose(np.array([[1.0, 1.0, 1.0]]), 5.0, 100.0)       # Q = 0: N* = 0 -> N = 1
    assert small["N"] == 1.0 and np.isclose(small["M"], 100.0 / 6.0)
    with pytest.raises(hs.HsimError):
        hs.oversim_cost_ratio(1.0, 1.0, 1.0, 64.0)
    with pytest.raises(hs.HsimError):
        hs.oversim_cost_ratio(1.0, 0.5, 1.0, 64.0)       # the larger n_b ran faster: P < 0
    with pytest.raises(hs.HsimError):
        hs.oversim_choose(mom, -1.0, 1e9)


def test_regression_rejects_misaligned_model(hs, cpu_only):
    """The BF16 kernel reads a network's weights in 8-byte pairs: a model pointer that is not
    8-byte aligned is refused before any launch (the FP32 / FP64 form takes any alignment)."""
    mlp = wl.MLPConfig(hidden=2, width=32, epochs=1, batch=64)
    cfg = hs.mlp_cfg(mlp, 3, 128)
    dates = np.array([1], dtype=np.int32)
    ok = ctypes.c_void_p(4096)
    odd = ctypes.c_void_p(4096 + 4)      # never dereferenced: validation fails first
    L = hs.lib()
    rc = L.cva_regress_fit(ctypes.byref(cfg), 1, dates.ctypes.data_as(hs._c_i32p), 3, 128, 3, ok, ok, None, 0,
                           odd, None, ok, 1 << 20, None)
    assert rc == -1 and "8-byte" in L.hsim_last_error().decode()
    rc = L.cva_regress_predict(ctypes.byref(cfg), 1, dates.ctypes.data_as(hs._c_i32p), 3, 128, 3, ok, odd, ok, None)
    assert rc == -1 and "8-byte" in L.hsim_last_error().decode()


def test_regression_rejects_unknown_tiling(hs, cpu_only):
    """cva_mlp_cfg.tile: the BF16 kernels' wave tilings 0 .. 2; the FP32 / FP64 form has only 0."""
    mlp = wl.MLPConfig(hidden=2, width=32, epochs=1, batch=64)
    dates = np.array([1], dtype=np.int32)
    ok = ctypes.c_void_p(4096)
    L = hs.lib()
    for tile, dtype in ((3, hs.REG_BF16), (-1, hs.REG_BF16), (1, hs.REG_FP32)):
        cfg = hs.mlp_cfg(mlp, 3, 128, dtype=dtype, tile=tile)
        rc = L.cva_regress_fit(ctypes.byref(cfg), 1, dates.ctypes.data_as(hs._c_i32p), 3, 128, 3, ok, ok, None, 0,
                               ok, None, ok, 1 << 20, None)
        assert rc == -2 and b"tile" in L.hsim_last_error()
