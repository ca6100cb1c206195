"""Python binding of libhsim (the C ABI declared in include/hsim.h).

Argument marshalling only: host parameters go into the C structs, device buffers are
torch tensors whose pointers are passed through, and every step of the computation runs
in the library's HIP kernels on the current torch stream.  There is no fallback: if the
library is not built, or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhsim.so")

HSIM_FP64, HSIM_FP32, HSIM_FP32_PLAIN = 0, 1, 2
REG_BF16, REG_FP32, REG_FP64 = 0, 1, 2
FEAT_FACTORS, FEAT_FACTORS_PLUS = 0, 1
OP_INNER, OP_TARGETS, OP_FUSED, OP_ADJOINT, OP_BRANCH, OP_FUSED_LAUNCH = 1, 2, 3, 4, 5, 6
HSIM_EINVAL, HSIM_ERANGE, HSIM_ENOWS, HSIM_EDEVICE, HSIM_EUNSUPPORTED, HSIM_ETIMEOUT = -1, -2, -3, -4, -5, -6

_c_i32p = ctypes.POINTER(ctypes.c_int32)
_c_f64p = ctypes.POINTER(ctypes.c_double)


class HsimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hsim error {code}: {msg}")
        self.code = code


class Market(ctypes.Structure):
    _fields_ = [("n_ccy", ctypes.c_int32), ("n_cpty", ctypes.c_int32),
                ("a", _c_f64p), ("b", _c_f64p), ("sigma_r", _c_f64p), ("r0", _c_f64p),
                ("sigma_fx", _c_f64p), ("fx0", _c_f64p), ("corr", _c_f64p),
                ("kappa", _c_f64p), ("theta", _c_f64p), ("nu", _c_f64p),
                ("lambda0", _c_f64p), ("lgd", _c_f64p)]


class Portfolio(ctypes.Structure):
    _fields_ = [("n_swaps", ctypes.c_int32), ("ccy", _c_i32p), ("cpty", _c_i32p),
                ("periods", _c_i32p), ("notional", _c_f64p), ("fixed_rate", _c_f64p),
                ("payer", _c_i32p), ("delta", ctypes.c_double)]


class MlpCfg(ctypes.Structure):
    _fields_ = [("hidden", ctypes.c_int32), ("width", ctypes.c_int32), ("d_in", ctypes.c_int32),
                ("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("warm_start", ctypes.c_int32), ("init_tag", ctypes.c_int32),
                ("team", ctypes.c_int32), ("dtype", ctypes.c_int32), ("tile", ctypes.c_int32)]


class Grid(ctypes.Structure):
    _fields_ = [("horizon", ctypes.c_double), ("n_dates", ctypes.c_int32),
                ("n_sub", ctypes.c_int32)]


_lib = None


def lib():
    """Load libhsim.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2211_17005_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, i64, u32, u64 = (ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32,
                                  ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64)
    M_, P_, G_ = ctypes.POINTER(Market), ctypes.POINTER(Portfolio), ctypes.POINTER(Grid)
    sig = {
        "hsim_abi_version": (ctypes.c_int, []),
        "hsim_last_error": (ctypes.c_char_p, []),
        "hsim_n_features": (ctypes.c_int, [M_, ctypes.c_int]),
        "hsim_par_rates": (ctypes.c_int, [M_, P_, _c_f64p]),
        "hsim_philox_fill": (ctypes.c_int, [u64, u32, u32, u32, i64, i64, vp, vp]),
        "hsim_normals_fill": (ctypes.c_int, [u64, i64, i64, i32, i32, ctypes.c_int, vp, vp]),
        "hsim_outer_paths": (ctypes.c_int, [M_, P_, G_, u64, i64, i64, ctypes.c_int, ctypes.c_int,
                                            vp, vp, vp, vp, vp, vp]),
        "hsim_inner_defaults": (ctypes.c_int, [G_, i32, u64, i64, i64, i32, vp, i32, vp, vp, vp,
                                               sz, vp]),
        "hsim_targets_cva": (ctypes.c_int, [G_, i32, i64, i32, vp, i32, ctypes.c_int, vp, vp, vp,
                                            vp, vp, vp, sz, vp]),
        "hsim_targets_cva_noalloc": (ctypes.c_int, [G_, i32, i64, i32, vp, i32, ctypes.c_int, vp, vp,
                                                    vp, vp, vp, vp]),
        "hsim_targets_intensity": (ctypes.c_int, [G_, i32, i64, ctypes.c_int, vp, vp, vp, vp, vp,
                                                  vp, sz, vp]),
        "hsim_inner_defaults_cva": (ctypes.c_int, [M_, P_, G_, u64, i64, i64, i32, vp, i32,
                                                   ctypes.c_int, ctypes.c_int, vp, vp, vp, vp, sz,
                                                   vp]),
        "hsim_workspace_bytes": (sz, [ctypes.c_int, M_, G_, i64, ctypes.c_int]),
        "hsim_fused": (ctypes.c_int, [M_, P_, G_, u64, i64, i64, i32, vp, i32, ctypes.c_int, ctypes.c_int,
                                      vp, vp, vp, vp, sz, vp]),
        "hsim_fused_keep": (ctypes.c_int, [M_, P_, G_, u64, i64, i64, i32, vp, i32, ctypes.c_int, ctypes.c_int,
                                           vp, vp, vp, i64, vp, vp, vp, vp, sz, vp]),
        "hsim_n_params": (ctypes.c_int, [M_]),
        "cva_adjoint": (ctypes.c_int, [M_, P_, G_, u64, i64, i64, vp, vp, vp, sz, vp]),
        "cva_regress_record_floats": (ctypes.c_int, [ctypes.POINTER(MlpCfg)]),
        "cva_regress_param_floats": (ctypes.c_int, [ctypes.POINTER(MlpCfg)]),
        "cva_regress_workspace_bytes": (sz, [ctypes.POINTER(MlpCfg), i32, i64]),
        "cva_regress_fit": (ctypes.c_int, [ctypes.POINTER(MlpCfg), i32, _c_i32p, i32, i64, i32, vp,
                                           vp, vp, u64, vp, vp, vp, sz, vp]),
        "hsim_sample_rows": (ctypes.c_int, [G_, i32, i32, u64, i64, i64, i32, ctypes.c_int, vp, vp, vp,
                                            vp, vp, vp, vp]),
        "hsim_targets_alive": (ctypes.c_int, [G_, i64, i32, vp, i32, ctypes.c_int, vp, vp, vp, vp, vp,
                                              vp, vp, sz, vp]),
        "cva_regress_predict": (ctypes.c_int, [ctypes.POINTER(MlpCfg), i32, _c_i32p, i32, i64, i32,
                                               vp, vp, vp, vp]),
        "hsim_oversim_moments": (ctypes.c_int, [G_, i64, ctypes.c_int, vp, vp, vp, vp, vp]),
        "hsim_branch_cva": (ctypes.c_int, [M_, P_, G_, u64, i64, i64, i32, i32, ctypes.c_int, vp, vp]),
        "hsim_branch_errors": (ctypes.c_int, [i64, i32, ctypes.c_int, vp, vp, vp, vp, sz, vp]),
        "cva_adjoint_forward": (ctypes.c_int, [M_, P_, G_, u64, i64, i64, i64, i32, vp, vp, vp, vp, vp,
                                               vp, vp, sz, vp]),
        "cva_regress_adam_state": (ctypes.c_int, [ctypes.POINTER(MlpCfg), i32, i64, vp, sz, vp, vp, vp, vp]),
        "hsim_set_wait_limit": (ctypes.c_int, [i32]),
        "hsim_oversim_cost_ratio": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                   ctypes.c_double, _c_f64p]),
        "hsim_oversim_choose": (ctypes.c_int, [i32, _c_f64p, ctypes.c_double, ctypes.c_double, _c_f64p,
                                               _c_f64p, _c_f64p, _c_f64p, _c_f64p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    _register_extra(L)
    return L


_extra_registrars = []


def _register_extra(L):
    for f in _extra_registrars:
        f(L)


def check(rc: int):
    if rc != 0:
        raise HsimError(rc, lib().hsim_last_error().decode())


# ------------------------------------------------------------------------------- marshalling
def _f64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))


def _i32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int32).reshape(-1))


def _ptr(arr, ctype):
    return arr.ctypes.data_as(ctypes.POINTER(ctype)) if arr.size else None


@dataclass
class _Keep:
    struct: ctypes.Structure
    arrays: list


def market_struct(m) -> _Keep:
    arrs = [_f64(getattr(m, f)) for f in ("a", "b", "sigma_r", "r0", "sigma_fx", "fx0", "corr",
                                          "kappa", "theta", "nu", "lambda0", "lgd")]
    s = Market(int(arrs[0].size), int(arrs[7].size), *[_ptr(a, ctypes.c_double) for a in arrs])
    return _Keep(s, arrs)


def portfolio_struct(book, fixed_rate) -> _Keep:
    delta = float(getattr(book, "delta", 1.0))
    periods = np.rint(np.asarray(book.maturity, dtype=np.float64) / delta).astype(np.int32)
    arrs = [_i32(book.ccy), _i32(book.cpty), _i32(periods), _f64(book.notional),
            _f64(fixed_rate), _i32(book.payer)]
    s = Portfolio(int(arrs[0].size), _ptr(arrs[0], ctypes.c_int32), _ptr(arrs[1], ctypes.c_int32),
                  _ptr(arrs[2], ctypes.c_int32), _ptr(arrs[3], ctypes.c_double),
                  _ptr(arrs[4], ctypes.c_double), _ptr(arrs[5], ctypes.c_int32), delta)
    return _Keep(s, arrs)


def grid_struct(g) -> Grid:
    return Grid(float(g.horizon), int(g.n_dates), int(g.n_sub))


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t):
    """Device pointer of a tensor; the C ABI takes dense row-major arrays only."""
    if t is None:
        return ctypes.c_void_p(0)
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("libhsim takes contiguous device tensors "
                         f"(got device={t.device}, strides={tuple(t.stride())})")
    return ctypes.c_void_p(t.data_ptr())


def _expect(t, dtype, shape, name):
    if t.dtype != dtype or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected {dtype} {tuple(shape)}, got {t.dtype} {tuple(t.shape)}")


def _real(precision):
    import torch
    return torch.float64 if precision == HSIM_FP64 else torch.float32


# ------------------------------------------------------------------------------- entry points
def abi_version() -> int:
    return lib().hsim_abi_version()


def n_features(market, feature_mode: int) -> int:
    k = market_struct(market)
    n = lib().hsim_n_features(ctypes.byref(k.struct), feature_mode)
    if n < 0:
        check(n)
    return n


def par_rates(market, book) -> np.ndarray:
    km = market_struct(market)
    kp = portfolio_struct(book, np.zeros(len(book.ccy)))
    out = np.zeros(len(book.ccy))
    check(lib().hsim_par_rates(ctypes.byref(km.struct), ctypes.byref(kp.struct),
                               out.ctypes.data_as(_c_f64p)))
    return out


def fixed_rates(market, book) -> np.ndarray:
    """Fixed rates of a book given as spreads over the time-0 par rate (library pricing)."""
    if getattr(book, "fixed_rate", None) is not None:
        return _f64(book.fixed_rate)
    return par_rates(market, book) + 1e-4 * _f64(book.spread_bp)


def philox_fill(seed: int, c1: int, c2: int, c3: int, k_begin: int, count: int):
    import torch
    out = torch.empty(4 * count, dtype=torch.int32, device="cuda")
    check(lib().hsim_philox_fill(seed, c1, c2, c3, k_begin, count, _dptr(out), _stream()))
    return out


def normals_fill(seed: int, path_begin: int, count: int, step: int, n_z: int, precision: int):
    import torch
    out = torch.empty((count, n_z), dtype=_real(precision), device="cuda")
    check(lib().hsim_normals_fill(seed, path_begin, count, step, n_z, precision, _dptr(out),
                                  _stream()))
    return out


def feature_mode_of(w) -> int:
    return FEAT_FACTORS_PLUS if getattr(w, "features", "factors") == "factors_plus" else FEAT_FACTORS


def outer_paths(w, precision: int = HSIM_FP32, path_begin: int = 0, M: Optional[int] = None,
                fixed=None, want_features=True, want_mtm=False, market=None):
    """hsim_outer_paths on a workload; returns dict of device tensors."""
    import torch
    m = w.market if market is None else market
    M = w.M if M is None else M
    n1 = w.grid.n_dates + 1
    C = m.n_cpty
    fm = feature_mode_of(w)
    d = n_features(m, fm)
    R = _real(precision)
    out = {
        "features": torch.empty((n1, d, M), dtype=R, device="cuda") if want_features else None,
        "I": torch.empty((n1, M), dtype=torch.float64, device="cuda"),
        "Lam": torch.empty((n1, C, M), dtype=torch.float64, device="cuda"),
        "D": torch.empty((n1, C, M), dtype=R, device="cuda"),
        "MtM": torch.empty((n1, C, M), dtype=R, device="cuda") if want_mtm else None,
    }
    fixed = fixed_rates(m, w.portfolio) if fixed is None else fixed
    km, kp = market_struct(m), portfolio_struct(w.portfolio, fixed)
    g = grid_struct(w.grid)
    check(lib().hsim_outer_paths(ctypes.byref(km.struct), ctypes.byref(kp.struct), ctypes.byref(g),
                                 w.seed, path_begin, M, precision, fm, _dptr(out["features"]),
                                 _dptr(out["I"]), _dptr(out["Lam"]), _dptr(out["D"]),
                                 _dptr(out["MtM"]), _stream()))
    return out


def _nb_args(n_b, n_b_per_block, block_paths):
    import torch
    if n_b_per_block is None:
        return int(n_b), None, 64
    t = torch.as_tensor(np.asarray(n_b_per_block, dtype=np.int32), device="cuda")
    return 0, t, int(block_paths)


def inner_defaults(grid, n_cpty: int, seed: int, Lam, path_begin: int = 0, n_b: int = 1,
                   n_b_per_block=None, block_paths: int = 64):
    import torch
    M = Lam.shape[-1]
    _expect(Lam, torch.float64, (grid.n_dates + 1, n_cpty, M), "Lambda")
    counts = torch.empty((grid.n_dates + 1, n_cpty, M), dtype=torch.int32, device="cuda")
    nb, nbt, bp = _nb_args(n_b, n_b_per_block, block_paths)
    g = grid_struct(grid)
    wsb = lib().hsim_workspace_bytes(OP_INNER, None, ctypes.byref(g), M, HSIM_FP32)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda") if nbt is not None else None
    check(lib().hsim_inner_defaults(ctypes.byref(g), n_cpty, seed, path_begin, M, nb, _dptr(nbt), bp,
                                    _dptr(Lam), _dptr(counts), _dptr(ws), wsb if ws is not None else 0,
                                    _stream()))
    torch.cuda.current_stream().synchronize() if nbt is not None else None
    return counts


def targets_cva(grid, n_cpty: int, I, D, counts, n_b: int = 1, n_b_per_block=None,
                block_paths: int = 64, precision: int = HSIM_FP32):
    import torch
    M = I.shape[-1]
    _expect(I, torch.float64, (grid.n_dates + 1, M), "I")
    _expect(D, _real(precision), (grid.n_dates + 1, n_cpty, M), "D")
    _expect(counts, torch.int32, (grid.n_dates + 1, n_cpty, M), "counts")
    T = torch.empty((grid.n_dates + 1, M), dtype=_real(precision), device="cuda")
    cva0 = torch.empty(1, dtype=torch.float64, device="cuda")
    g = grid_struct(grid)
    wsb = lib().hsim_workspace_bytes(OP_TARGETS, None, ctypes.byref(g), M, precision)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
    nb, nbt, bp = _nb_args(n_b, n_b_per_block, block_paths)
    check(lib().hsim_targets_cva(ctypes.byref(g), n_cpty, M, nb, _dptr(nbt), bp, precision,
                                 _dptr(I), _dptr(D), _dptr(counts), _dptr(T), _dptr(cva0),
                                 _dptr(ws), wsb, _stream()))
    torch.cuda.current_stream().synchronize() if nbt is not None else None
    return T, cva0


def targets_cva_noalloc(grid, n_cpty: int, I, D, counts, n_b: int = 1, n_b_per_block=None,
                        block_paths: int = 64, precision: int = HSIM_FP32):
    """hsim_targets_cva_noalloc: targets_cva without a workspace (the library's static scratch)."""
    import torch
    M = I.shape[-1]
    _expect(I, torch.float64, (grid.n_dates + 1, M), "I")
    _expect(D, _real(precision), (grid.n_dates + 1, n_cpty, M), "D")
    _expect(counts, torch.int32, (grid.n_dates + 1, n_cpty, M), "counts")
    T = torch.empty((grid.n_dates + 1, M), dtype=_real(precision), device="cuda")
    cva0 = torch.empty(1, dtype=torch.float64, device="cuda")
    g = grid_struct(grid)
    nb, nbt, bp = _nb_args(n_b, n_b_per_block, block_paths)
    check(lib().hsim_targets_cva_noalloc(ctypes.byref(g), n_cpty, M, nb, _dptr(nbt), bp, precision,
                                         _dptr(I), _dptr(D), _dptr(counts), _dptr(T), _dptr(cva0),
                                         _stream()))
    torch.cuda.current_stream().synchronize() if nbt is not None else None
    return T, cva0


def sample_rows(w, out, n_b: Optional[int] = None, precision: int = HSIM_FP32, path_begin: int = 0):
    """hsim_sample_rows on the outputs `out` of outer_paths (same precision and path range):
    X [n+1][d + C][n_b M], Y [n+1][n_b M] float32 device tensors."""
    import torch
    n_b = w.n_b if n_b is None else n_b
    I = out["I"]
    n1, M = I.shape
    C = out["Lam"].shape[1]
    feats = out["features"]
    d = 0 if feats is None else int(feats.shape[1])
    X = torch.empty((n1, d + C, n_b * M), dtype=torch.float32, device="cuda")
    Y = torch.empty((n1, n_b * M), dtype=torch.float32, device="cuda")
    g = grid_struct(w.grid)
    check(lib().hsim_sample_rows(ctypes.byref(g), C, d, w.seed, path_begin, M, n_b, precision,
                                 _dptr(feats), _dptr(I), _dptr(out["Lam"]), _dptr(out["D"]), _dptr(X),
                                 _dptr(Y), _stream()))
    return X, Y


def targets_alive(grid, I, D, counts, n_b: int = 1, n_b_per_block=None, block_paths: int = 64,
                  precision: int = HSIM_FP32):
    """hsim_targets_alive (one counterparty): the alive-group targets, their weights and CVA_0."""
    import torch
    M = I.shape[-1]
    _expect(I, torch.float64, (grid.n_dates + 1, M), "I")
    _expect(D, _real(precision), (grid.n_dates + 1, 1, M), "D")
    _expect(counts, torch.int32, (grid.n_dates + 1, 1, M), "counts")
    T = torch.empty((grid.n_dates + 1, M), dtype=_real(precision), device="cuda")
    Wt = torch.empty((grid.n_dates + 1, M), dtype=torch.float32, device="cuda")
    cva0 = torch.empty(1, dtype=torch.float64, device="cuda")
    g = grid_struct(grid)
    wsb = lib().hsim_workspace_bytes(OP_TARGETS, None, ctypes.byref(g), M, precision)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
    nb, nbt, bp = _nb_args(n_b, n_b_per_block, block_paths)
    check(lib().hsim_targets_alive(ctypes.byref(g), M, nb, _dptr(nbt), bp, precision, _dptr(I),
                                   _dptr(D), _dptr(counts), _dptr(T), _dptr(Wt), _dptr(cva0),
                                   _dptr(ws), wsb, _stream()))
    torch.cuda.current_stream().synchronize() if nbt is not None else None
    return T, Wt, cva0


def targets_intensity(grid, n_cpty: int, I, Lam, D, precision: int = HSIM_FP32):
    """hsim_targets_intensity: the conditional-expectation targets (no inner draws) and CVA_0."""
    import torch
    M = I.shape[-1]
    _expect(I, torch.float64, (grid.n_dates + 1, M), "I")
    _expect(Lam, torch.float64, (grid.n_dates + 1, n_cpty, M), "Lam")
    _expect(D, _real(precision), (grid.n_dates + 1, n_cpty, M), "D")
    T = torch.empty((grid.n_dates + 1, M), dtype=_real(precision), device="cuda")
    cva0 = torch.empty(1, dtype=torch.float64, device="cuda")
    g = grid_struct(grid)
    wsb = lib().hsim_workspace_bytes(OP_TARGETS, None, ctypes.byref(g), M, precision)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
    check(lib().hsim_targets_intensity(ctypes.byref(g), n_cpty, M, precision, _dptr(I), _dptr(Lam),
                                       _dptr(D), _dptr(T), _dptr(cva0), _dptr(ws), wsb, _stream()))
    return T, cva0


BRANCH_STATS = ("cva_mean", "cva_sq_nested", "cva_sq", "mse_nested", "mse_twin", "phi_mean")


def branch_cva(w, date: int, n_branch: int, precision: int = HSIM_FP32, path_begin: int = 0,
               M: Optional[int] = None, fixed=None, market=None):
    """hsim_branch_cva: xi [n_branch][M] (float64, device), the eq. CVAint samples of
    n_branch continuations of every path after pricing date `date`."""
    import torch
    m = w.market if market is None else market
    M = w.M if M is None else M
    xi = torch.empty((n_branch, M), dtype=torch.float64, device="cuda")
    fixed = fixed_rates(m, w.portfolio) if fixed is None else fixed
    km, kp = market_struct(m), portfolio_struct(w.portfolio, fixed)
    g = grid_struct(w.grid)
    check(lib().hsim_branch_cva(ctypes.byref(km.struct), ctypes.byref(kp.struct), ctypes.byref(g),
                                w.seed, path_begin, M, date, n_branch, precision, _dptr(xi),
                                _stream()))
    return xi


def branch_errors(xi, phi=None) -> dict:
    """hsim_branch_errors: nested / twin Monte Carlo statistics (names in BRANCH_STATS) of the
    prediction phi [M] (float32 or float64 device tensor, or None for phi = 0)."""
    import torch
    B, M = xi.shape
    _expect(xi, torch.float64, (B, M), "xi")
    precision = HSIM_FP64
    if phi is not None:
        precision = HSIM_FP32 if phi.dtype == torch.float32 else HSIM_FP64
        _expect(phi, _real(precision), (M,), "phi")
    out = torch.empty(len(BRANCH_STATS), dtype=torch.float64, device="cuda")
    wsb = lib().hsim_workspace_bytes(OP_BRANCH, None, None, M, precision)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
    check(lib().hsim_branch_errors(M, B, precision, _dptr(phi), _dptr(xi), _dptr(out), _dptr(ws),
                                   wsb, _stream()))
    return dict(zip(BRANCH_STATS, out.cpu().tolist()))


def oversim_moments(grid, T1, T2, pred=None, precision: int = HSIM_FP32):
    """hsim_oversim_moments: [n+1][3] = E[g], E[g^2], E[g g'] of the two pilot continuations."""
    import torch
    M = T1.shape[-1]
    R = _real(precision)
    _expect(T1, R, (grid.n_dates + 1, M), "T1")
    _expect(T2, R, (grid.n_dates + 1, M), "T2")
    if pred is not None:
        _expect(pred, R, (grid.n_dates + 1, M), "pred")
    out = torch.empty((grid.n_dates + 1, 3), dtype=torch.float64, device="cuda")
    g = grid_struct(grid)
    check(lib().hsim_oversim_moments(ctypes.byref(g), M, precision, _dptr(T1), _dptr(T2), _dptr(pred),
                                     _dptr(out), _stream()))
    return out


def oversim_cost_ratio(t: float, t_prime: float, N: float, N_prime: float) -> float:
    """hsim_oversim_cost_ratio: P from two timings (l:ratio)."""
    P = ctypes.c_double(0.0)
    check(lib().hsim_oversim_cost_ratio(float(t), float(t_prime), float(N), float(N_prime), ctypes.byref(P)))
    return P.value


def oversim_choose(moments, P: float, Psi: float) -> dict:
    """hsim_oversim_choose on host moments [n+1][3]: R, Q, N*_i (NaN where undefined), N, M."""
    mom = np.ascontiguousarray(np.asarray(moments, dtype=np.float64))
    n1 = int(mom.shape[0])
    R, Q, Ns = np.empty(n1), np.empty(n1), np.empty(n1)
    N, Mo = ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = lib().hsim_oversim_choose(n1, mom.ctypes.data_as(_c_f64p), float(P), float(Psi),
                                   R.ctypes.data_as(_c_f64p), Q.ctypes.data_as(_c_f64p),
                                   Ns.ctypes.data_as(_c_f64p), ctypes.byref(N), ctypes.byref(Mo))
    if rc < 0:
        check(rc)
    return {"R": R, "Q": Q, "N_dates": Ns, "N": N.value, "M": Mo.value, "defined": rc}


def workspace_bytes(op: int, w, M: int, precision: int) -> int:
    km = market_struct(w.market)
    g = grid_struct(w.grid)
    return int(lib().hsim_workspace_bytes(op, ctypes.byref(km.struct), ctypes.byref(g), M, precision))


class Solver:
    """Holds the marshalled parameters and workspace of one workload for repeated calls."""

    def __init__(self, w, precision: int = HSIM_FP32, M: Optional[int] = None, fixed=None,
                 n_b_per_block=None, block_paths: int = 64, market=None):
        import torch
        self.w = w
        self.market = w.market if market is None else market
        self.precision = precision
        self.M = w.M if M is None else M
        self.fixed = fixed_rates(self.market, w.portfolio) if fixed is None else fixed
        self.km = market_struct(self.market)
        self.kp = portfolio_struct(w.portfolio, self.fixed)
        self.g = grid_struct(w.grid)
        self.fm = feature_mode_of(w)
        self.d = n_features(self.market, self.fm)
        self.nb, self.nbt, self.bp = _nb_args(w.n_b, n_b_per_block, block_paths)
        wsb = lib().hsim_workspace_bytes(OP_FUSED, ctypes.byref(self.km.struct),
                                         ctypes.byref(self.g), self.M, precision)
        self.wsb = wsb
        self.ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        R = _real(precision)
        n1 = w.grid.n_dates + 1
        self.features = torch.empty((n1, self.d, self.M), dtype=R, device="cuda")
        self.T = torch.empty((n1, self.M), dtype=R, device="cuda")
        self.cva0 = torch.empty(1, dtype=torch.float64, device="cuda")

    def inner_defaults_cva(self, path_begin: int = 0, want_features: bool = True):
        check(lib().hsim_inner_defaults_cva(
            ctypes.byref(self.km.struct), ctypes.byref(self.kp.struct), ctypes.byref(self.g),
            self.w.seed, path_begin, self.M, self.nb, _dptr(self.nbt), self.bp, self.precision,
            self.fm, _dptr(self.features if want_features else None), _dptr(self.T),
            _dptr(self.cva0), _dptr(self.ws), self.wsb, _stream()))
        return self.features, self.T, self.cva0


class FusedSolver(Solver):
    """hsim_fused: the whole simulation in one launch (same outputs as Solver.inner_defaults_cva)."""

    def __init__(self, w, precision: int = HSIM_FP32, M: Optional[int] = None, fixed=None,
                 n_b_per_block=None, block_paths: int = 64, market=None):
        import torch
        super().__init__(w, precision, M, fixed, n_b_per_block, block_paths, market)
        self.wsb = lib().hsim_workspace_bytes(OP_FUSED_LAUNCH, ctypes.byref(self.km.struct),
                                              ctypes.byref(self.g), self.M, precision)
        self.ws = torch.empty(self.wsb, dtype=torch.uint8, device="cuda")

    def run(self, path_begin: int = 0, want_features: bool = True):
        check(lib().hsim_fused(
            ctypes.byref(self.km.struct), ctypes.byref(self.kp.struct), ctypes.byref(self.g),
            self.w.seed, path_begin, self.M, self.nb, _dptr(self.nbt), self.bp, self.precision,
            self.fm, _dptr(self.features if want_features else None), _dptr(self.T),
            _dptr(self.cva0), _dptr(self.ws), self.wsb, _stream()))
        return self.features, self.T, self.cva0

    def run_keep(self, n_keep: int, I, Lam, D, path_begin: int = 0, want_features: bool = True):
        """hsim_fused_keep: run() plus the forward states of the first n_keep paths into I [n+1][M],
        Lam [n+1][C][M] (float64) and D [n+1][C][M] (the solver's real type)."""
        import torch
        n1, C = self.w.grid.n_dates + 1, self.market.n_cpty
        _expect(I, torch.float64, (n1, self.M), "I")
        _expect(Lam, torch.float64, (n1, C, self.M), "Lambda")
        _expect(D, _real(self.precision), (n1, C, self.M), "D")
        check(lib().hsim_fused_keep(
            ctypes.byref(self.km.struct), ctypes.byref(self.kp.struct), ctypes.byref(self.g),
            self.w.seed, path_begin, self.M, self.nb, _dptr(self.nbt), self.bp, self.precision,
            self.fm, _dptr(self.features if want_features else None), _dptr(self.T),
            _dptr(self.cva0), int(n_keep), _dptr(I), _dptr(Lam), _dptr(D), _dptr(self.ws), self.wsb, _stream()))
        return self.features, self.T, self.cva0


def inner_defaults_cva(w, precision: int = HSIM_FP32, path_begin: int = 0, M=None,
                       n_b_per_block=None, block_paths: int = 64):
    s = Solver(w, precision, M, n_b_per_block=n_b_per_block, block_paths=block_paths)
    return s.inner_defaults_cva(path_begin)


# ------------------------------------------------------------------------------- regression
def mlp_cfg(mlp, d_in: int, M: int, warm_start: bool = False, init_tag: int = 0,
            team: int = 0, dtype: int = REG_BF16, tile: int = 0) -> MlpCfg:
    """C config from a workload's MLP settings (batch = M / n_batches when no batch is given);
    team = workgroups per date (0: the library's choice); dtype REG_BF16 / REG_FP32 / REG_FP64;
    tile = the BF16 kernels' wave tiling variant (0, 1, 2)."""
    batch = int(mlp.batch) if getattr(mlp, "batch", None) else max(1, M // int(mlp.n_batches))
    return MlpCfg(int(mlp.hidden), int(mlp.width), int(d_in), int(mlp.epochs), batch,
                  float(mlp.lr), float(mlp.beta1), float(mlp.beta2), float(mlp.eps),
                  1 if warm_start else 0, int(init_tag), int(team), int(dtype), int(tile))

MLP_TILES = 3


def reg_dtype(cfg: MlpCfg):
    """torch element type of a fit's inputs, model and losses."""
    import torch
    return torch.float64 if cfg.dtype == REG_FP64 else torch.float32


def record_floats(cfg: MlpCfg) -> int:
    n = lib().cva_regress_record_floats(ctypes.byref(cfg))
    if n < 0:
        check(n)
    return n


def regress_fit(cfg: MlpCfg, dates, X, Y, seed: int = 0, want_loss: bool = True, W=None):
    """cva_regress_fit: X [n+1][n_feat][M], Y [n+1][M], W [n+1][M] row weights or None (device;
    float32, or float64 for REG_FP64)."""
    import torch
    n1, n_feat, M = X.shape
    R = reg_dtype(cfg)
    _expect(Y, R, (n1, M), "Y")
    _expect(X, R, (n1, n_feat, M), "X")
    if W is not None:
        _expect(W, R, (n1, M), "W")
    d = _i32(dates)
    n_reg = int(d.size)
    rec = record_floats(cfg)
    model = torch.zeros((n_reg, rec), dtype=R, device="cuda")
    loss = torch.zeros((n_reg, cfg.epochs), dtype=R, device="cuda") if want_loss else None
    wsb = lib().cva_regress_workspace_bytes(ctypes.byref(cfg), n_reg, M)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    check(lib().cva_regress_fit(ctypes.byref(cfg), n_reg, d.ctypes.data_as(_c_i32p), n1, M, n_feat,
                                _dptr(X), _dptr(Y), _dptr(W), seed, _dptr(model), _dptr(loss), _dptr(ws), wsb,
                                _stream()))
    return model, loss, ws


def regress_adam_state(cfg: MlpCfg, n_reg: int, M: int, ws):
    """cva_regress_adam_state: (params, m, v) [n_reg][n_params] after a fit on workspace ws."""
    import torch
    L = lib()
    npar = L.cva_regress_param_floats(ctypes.byref(cfg))
    if npar < 0:
        check(npar)
    out = [torch.empty((n_reg, npar), dtype=reg_dtype(cfg), device="cuda") for _ in range(3)]
    check(L.cva_regress_adam_state(ctypes.byref(cfg), n_reg, M, _dptr(ws), ws.numel(), _dptr(out[0]),
                                   _dptr(out[1]), _dptr(out[2]), _stream()))
    return tuple(out)


def set_wait_limit(polls: int):
    """hsim_set_wait_limit: polls before the regression's bounded waits give up (0: default)."""
    check(lib().hsim_set_wait_limit(int(polls)))


def regress_predict(cfg: MlpCfg, dates, X, model):
    import torch
    n1, n_feat, M = X.shape
    d = _i32(dates)
    out = torch.empty((int(d.size), M), dtype=reg_dtype(cfg), device="cuda")
    check(lib().cva_regress_predict(ctypes.byref(cfg), int(d.size), d.ctypes.data_as(_c_i32p), n1, M,
                                    n_feat, _dptr(X), _dptr(model), _dptr(out), _stream()))
    return out


# ------------------------------------------------------------------------------- sensitivities
PARAM_FIELDS = ("r0", "fx0", "lambda0", "a", "b", "sigma_r", "sigma_fx", "kappa", "theta", "nu")


def n_params(market) -> int:
    k = market_struct(market)
    n = lib().hsim_n_params(ctypes.byref(k.struct))
    if n < 0:
        check(n)
    return n


class Adjoint:
    """Holds the workspace of cva_adjoint for one workload; call() returns (cva0, grad) tensors."""

    def __init__(self, w, M: Optional[int] = None, fixed=None):
        import torch
        self.w = w
        self.M = w.M if M is None else M
        self.fixed = fixed_rates(w.market, w.portfolio) if fixed is None else fixed
        self.kp = portfolio_struct(w.portfolio, self.fixed)
        self.g = grid_struct(w.grid)
        km = market_struct(w.market)
        self.wsb = lib().hsim_workspace_bytes(OP_ADJOINT, ctypes.byref(km.struct), ctypes.byref(self.g),
                                              self.M, HSIM_FP32)
        self.ws = torch.empty(self.wsb, dtype=torch.uint8, device="cuda")
        self.P = n_params(w.market)
        self.cva0 = torch.empty(1, dtype=torch.float64, device="cuda")
        self.grad = torch.empty(self.P, dtype=torch.float64, device="cuda")

    def from_forward(self, features, I, Lam, D, path_begin: int = 0, with_grad: bool = True):
        """cva_adjoint_forward on the first self.M paths of an earlier FP32 simulation of the same
        workload (features [n+1][d][ld], I [n+1][ld], Lam and D [n+1][C][ld] device tensors)."""
        km = market_struct(self.w.market)
        ld = int(I.shape[-1])
        check(lib().cva_adjoint_forward(ctypes.byref(km.struct), ctypes.byref(self.kp.struct),
                                        ctypes.byref(self.g), self.w.seed, path_begin, self.M, ld,
                                        int(features.shape[1]), _dptr(features), _dptr(I), _dptr(Lam),
                                        _dptr(D), _dptr(self.cva0),
                                        _dptr(self.grad if with_grad else None), _dptr(self.ws), self.wsb,
                                        _stream()))
        return self.cva0, self.grad

    def __call__(self, market=None, path_begin: int = 0, with_grad: bool = True):
        km = market_struct(self.w.market if market is None else market)
        check(lib().cva_adjoint(ctypes.byref(km.struct), ctypes.byref(self.kp.struct), ctypes.byref(self.g),
                                self.w.seed, path_begin, self.M, _dptr(self.cva0),
                                _dptr(self.grad if with_grad else None), _dptr(self.ws), self.wsb, _stream()))
        return self.cva0, self.grad


def pack_params(market) -> np.ndarray:
    return np.concatenate([np.asarray(getattr(market, f), dtype=np.float64).reshape(-1) for f in PARAM_FIELDS])


def unpack_params(market, vec):
    import dataclasses
    kw, o = {}, 0
    for f in PARAM_FIELDS:
        k = len(np.asarray(getattr(market, f)).reshape(-1))
        kw[f] = np.array(vec[o:o + k], dtype=np.float64)
        o += k
    return dataclasses.replace(market, **kw)


def cva_function():
    """torch.autograd.Function: CVA_0(params) with params a CPU float64 vector in the order of
    PARAM_FIELDS; backward uses the library's adjoint gradient."""
    import torch

    class CVA(torch.autograd.Function):
        @staticmethod
        def forward(ctx, params, adj):
            m = unpack_params(adj.w.market, params.detach().cpu().numpy())
            cva0, grad = adj(m)
            ctx.save_for_backward(grad.detach().cpu().clone())
            return cva0.detach().cpu().clone()[0]

        @staticmethod
        def backward(ctx, gout):
            (grad,) = ctx.saved_tensors
            return gout * grad, None

    return CVA
