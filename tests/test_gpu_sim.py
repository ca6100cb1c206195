"""Parity of the HIP simulation path (outer paths, inner defaults, targets, CVA_0) with the
FP64 oracle, through the C ABI.

Tolerances
  * RNG words, uniforms, default counts: bit-exact.
  * FP64 mode: 1e-12 relative (different operation order and libm only).
  * FP32 mode: 1e-5 relative for the simulation (state scale-relative; swap values and
    exposures relative to the gross notional of the netting set, because a swap value is a
    difference of two legs of notional size).  Default counts in FP32 mode must equal the
    counts the exact rule gives on the GPU's own Lambda; disagreements with the oracle can
    only come from draws within 1e-5 (relative) of a threshold and are counted and reported.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import inner as oinner
from oracle import model, philox, pipeline

pytestmark = pytest.mark.gpu


def npy(t):
    return t.detach().cpu().numpy()


def scale_err(got, ref):
    den = max(float(np.max(np.abs(ref))), 1e-300)
    return float(np.max(np.abs(got - ref))) / den


def gross_notional(w):
    g = np.zeros(w.market.n_cpty)
    fx = np.concatenate([[1.0], w.market.fx0])
    for s in range(w.portfolio.n_swaps):
        g[w.portfolio.cpty[s]] += w.portfolio.notional[s] * fx[w.portfolio.ccy[s]]
    return g


def rel(a, b):
    return abs(a - b) / abs(b) if b != 0 else abs(a)


def report(name, err, tol):
    print(f"  {name}: err vs FP64 = {err:.3e} (tol {tol:.0e})", flush=True)
    assert err <= tol, (name, err, tol)


# --------------------------------------------------------------------------------- RNG
def test_philox_words_bit_exact(lib):
    for (c1, c2, c3) in ((0, 0, 0), (17, 3, 0), (5, 0, 1), (9, 1, 2)):
        got = npy(lib.philox_fill(12345, c1, c2, c3, 1000, 1 << 16)).view(np.uint32)
        ref = philox.raw_words(12345, c1, c2, c3, 1000, 1 << 16)
        assert np.array_equal(got, ref)
    # the top of the counter range
    got = npy(lib.philox_fill((7 << 32) | 3, 1, 2, 3, (1 << 32) - 64, 64)).view(np.uint32)
    assert np.array_equal(got, philox.raw_words((7 << 32) | 3, 1, 2, 3, (1 << 32) - 64, 64))


@pytest.mark.parametrize("precision,tol", [(0, 1e-14), (1, 2e-6)])
def test_normals_match_oracle(lib, precision, tol):
    got = npy(lib.normals_fill(0, 100, 4096, 37, 27, precision)).astype(np.float64)
    ref = philox.outer_normals(0, np.arange(100, 100 + 4096), 37, 27)
    err = np.max(np.abs(got - ref) / np.maximum(1.0, np.abs(ref)))
    report(f"normals precision={precision}", err, tol)


# --------------------------------------------------------------------------------- outer
CASES = [
    ("plain", lambda: wl.plain_fp64().with_(M=1024)),
    ("small_multi", lambda: wl.small_multi(M=200)),          # ragged last tile
    ("tiny", lambda: wl.tiny(M=3)),
]


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def case(request):
    w = request.param[1]()
    ref = pipeline.simulate(w)
    return w, ref


@pytest.mark.parametrize("precision", [0, 1])
def test_outer_paths_match_oracle(lib, case, precision):
    w, ref = case
    out = lib.outer_paths(w, precision=precision, want_mtm=True)
    tol = 1e-12 if precision == 0 else 1e-5
    print(f"[{w.name} precision={precision}]")
    report("I", scale_err(npy(out["I"]), ref["I"]), tol)
    report("Lambda", scale_err(npy(out["Lam"]), ref["Lam"]), tol)
    F, Fr = npy(out["features"]).astype(np.float64), ref["features"]
    for f in range(F.shape[1]):
        report(f"feature {f}", scale_err(F[:, f], Fr[:, f]), tol)
    g = np.maximum(gross_notional(w), 1.0)[None, :, None]
    mt = npy(out["MtM"]).astype(np.float64)
    report("MtM / gross notional", float(np.max(np.abs(mt - ref["MtM"]) / g)), tol)
    D = npy(out["D"]).astype(np.float64)
    report("D / gross notional", float(np.max(np.abs(D - ref["D"]) / g)), tol)


def test_inner_counts_bit_exact_on_oracle_lambda(lib, case):
    """Fed the oracle's own Lambda, the GPU default counts equal the literal rule's."""
    import torch
    w, ref = case
    Lam = torch.as_tensor(ref["Lam"], device="cuda")
    cnt = npy(lib.inner_defaults(w.grid, w.market.n_cpty, w.seed, Lam, n_b=w.n_b))
    assert np.array_equal(cnt, ref["cnt"])


@pytest.mark.parametrize("precision", [0, 1])
def test_targets_and_cva0_match_oracle(lib, case, precision):
    w, ref = case
    feats, T, cva0 = lib.inner_defaults_cva(w, precision=precision)
    T = npy(T).astype(np.float64)
    out = lib.outer_paths(w, precision=precision, want_features=False)
    cnt = npy(lib.inner_defaults(w.grid, w.market.n_cpty, w.seed, out["Lam"], n_b=w.n_b))
    if precision == 0:
        assert np.array_equal(cnt, ref["cnt"])
        report("T", scale_err(T, ref["T"]), 1e-12)
        report("CVA_0", rel(cva0.item(), ref["cva0"]), 1e-12)
        return
    # FP32: the GPU's counts are the exact rule applied to the GPU's Lambda ...
    u = oinner.inner_draws(w, np.arange(w.M))
    Lg = np.transpose(npy(out["Lam"]), (0, 2, 1))
    js = oinner.default_dates(Lg, u)
    assert np.array_equal(cnt, oinner.default_counts(js, w.grid.n_dates))
    # ... and every disagreement with the oracle sits inside the guard band
    js_ref = oinner.default_dates(np.transpose(ref["Lam"], (0, 2, 1)), u)
    bad = np.argwhere(js != js_ref)
    eps = -np.log(u)
    Lr = np.transpose(ref["Lam"], (0, 2, 1))
    for (k, l, c) in bad:
        j = min(js[k, l, c], js_ref[k, l, c])
        lam = Lr[j, k, c]
        assert abs(lam - eps[k, l, c]) <= 1e-5 * max(lam, eps[k, l, c])
    print(f"  default draws differing from the oracle (all in the 1e-5 band): {len(bad)}")
    # T on every path: the oracle's recursion on its own I and MtM with the GPU's default dates
    mt = np.transpose(ref["MtM"], (0, 2, 1))
    T_js = oinner.targets(oinner.pathwise_loss(ref["I"], mt, w.market.lgd, js))
    report("T (all paths, GPU default dates)", scale_err(T, T_js), 1e-5)
    # CVA_0 on the GPU's default dates, and the bound on what the moved draws can change: one
    # draw moves its path's xi_0 by at most LGD_c max_i exp(-I_i) (MtM_c,i)^+, over n_b M
    report("CVA_0 (GPU default dates)", rel(cva0.item(), float(T_js[0].mean())), 1e-5)
    disc = np.exp(-ref["I"])[:, None, :] * np.maximum(ref["MtM"], 0.0)   # [n+1, C, M]
    pos_max = np.max(disc, axis=0)
    moved = sum(w.market.lgd[c] * pos_max[c, k] for (k, l, c) in bad) / (w.n_b * w.M)
    err = abs(cva0.item() - ref["cva0"])
    print(f"  CVA_0 |gpu - oracle| {err:.3e} <= 1e-5 |CVA_0| + {moved:.3e} (moved draws)", flush=True)
    assert err <= 1e-5 * abs(ref["cva0"]) + moved


def test_fused_equals_separate_stages(lib):
    w = wl.small_multi(M=333)
    for precision in (0, 1):
        f1, T1, c1 = lib.inner_defaults_cva(w, precision=precision)
        out = lib.outer_paths(w, precision=precision)
        cnt = lib.inner_defaults(w.grid, w.market.n_cpty, w.seed, out["Lam"], n_b=w.n_b)
        T2, c2 = lib.targets_cva(w.grid, w.market.n_cpty, out["I"], out["D"], cnt, n_b=w.n_b,
                                 precision=precision)
        assert np.array_equal(npy(f1), npy(out["features"]))
        assert np.array_equal(npy(T1), npy(T2))
        assert c1.item() == c2.item()


FUSED_CASES = [
    ("plain", lambda: wl.plain_fp64().with_(M=1000)),                 # ragged last tile
    ("small_multi", lambda: wl.small_multi(M=333, n_b=13)),           # n_b not a multiple of 4
    ("tiny", lambda: wl.tiny(M=3)),
    ("ten_currencies", lambda: wl.cva_at_scale(M=4096 + 17, n_b=128)),
]


@pytest.mark.parametrize("name", [c[0] for c in FUSED_CASES])
@pytest.mark.parametrize("precision", [0, 1])
def test_one_launch_equals_separate_stages(lib, name, precision):
    """hsim_fused (outer paths, inner draws and targets in one launch) gives the features, targets
    and CVA_0 of the separate stages bit for bit."""
    import torch
    w = dict(FUSED_CASES)[name]()
    if precision == 0 and name == "ten_currencies":
        w = w.with_(M=1024 + 5)
    s = lib.Solver(w, precision=precision)
    f1, T1, c1 = [x.clone() for x in s.inner_defaults_cva()]
    fs = lib.FusedSolver(w, precision=precision)
    f2, T2, c2 = fs.run()
    torch.cuda.synchronize()
    print(f"  [{w.name} precision {precision}] CVA_0 {c2.item():.12g}", flush=True)
    assert torch.equal(f1, f2) and torch.equal(T1, T2) and torch.equal(c1, c2)


@pytest.mark.parametrize("name", ["small_multi", "ten_currencies"])
def test_one_launch_keeps_forward_states(lib, name):
    """hsim_fused_keep writes I, Lambda and D of the first n_keep paths (ragged, not a whole tile)
    date-major exactly as hsim_outer_paths does, leaves the other columns alone, and changes
    nothing else of the one-launch results."""
    import torch
    w = dict(FUSED_CASES)[name]()
    M, n1, C = w.M, w.grid.n_dates + 1, w.market.n_cpty
    n_keep = M // 2 + 3
    out = lib.outer_paths(w, precision=1, want_features=False)
    fs = lib.FusedSolver(w, precision=1)
    f1, T1, c1 = [x.clone() for x in fs.run()]
    I = torch.full((n1, M), float("nan"), dtype=torch.float64, device="cuda")
    Lam = torch.full((n1, C, M), float("nan"), dtype=torch.float64, device="cuda")
    D = torch.full((n1, C, M), float("nan"), dtype=torch.float32, device="cuda")
    f2, T2, c2 = fs.run_keep(n_keep, I, Lam, D)
    torch.cuda.synchronize()
    assert torch.equal(f1, f2) and torch.equal(T1, T2) and torch.equal(c1, c2)
    assert torch.equal(I[:, :n_keep], out["I"][:, :n_keep])
    assert torch.equal(Lam[..., :n_keep], out["Lam"][..., :n_keep])
    assert torch.equal(D[..., :n_keep], out["D"][..., :n_keep])
    assert bool(torch.isnan(I[:, n_keep:]).all() and torch.isnan(Lam[..., n_keep:]).all()
                and torch.isnan(D[..., n_keep:]).all())


def test_one_launch_uneven_nb_and_path_offset(lib):
    """Uneven n_b per block of 64 paths and a path range that does not start at 0."""
    import torch
    w = wl.small_multi(M=640, n_b=8)
    levels = np.array([1, 8, 64, 3, 17, 2, 128, 5, 9, 33], dtype=np.int32)
    s = lib.Solver(w, precision=1, n_b_per_block=levels, block_paths=64)
    f1, T1, c1 = [x.clone() for x in s.inner_defaults_cva(path_begin=77)]
    fs = lib.FusedSolver(w, precision=1, n_b_per_block=levels, block_paths=64)
    f2, T2, c2 = fs.run(path_begin=77)
    torch.cuda.synchronize()
    assert torch.equal(f1, f2) and torch.equal(T1, T2) and torch.equal(c1, c2)


def test_deterministic_and_split_invariant(lib):
    """Two runs agree bitwise; simulating [0, M/2) and [M/2, M) separately changes nothing."""
    w = wl.small_multi(M=256)
    f1, T1, _ = [x.clone() for x in lib.inner_defaults_cva(w, precision=1)]
    f2, T2, _ = lib.inner_defaults_cva(w, precision=1)
    assert np.array_equal(npy(f1), npy(f2)) and np.array_equal(npy(T1), npy(T2))
    half = w.M // 2
    fa, Ta, _ = [x.clone() for x in lib.inner_defaults_cva(w, precision=1, path_begin=0, M=half)]
    fb, Tb, _ = lib.inner_defaults_cva(w, precision=1, path_begin=half, M=w.M - half)
    assert np.array_equal(np.concatenate([npy(Ta), npy(Tb)], axis=1), npy(T1))
    assert np.array_equal(np.concatenate([npy(fa), npy(fb)], axis=2), npy(f1))


def test_uneven_oversimulation_matches_oracle(lib):
    w = wl.oversim_sweep(M=640, levels=(1, 8, 64, 5, 1024))
    nbb = w.extra["n_b_per_block"]
    nbp = np.repeat(nbb, 64)[:w.M]
    ref = pipeline.simulate(w, n_b_per_path=nbp)
    _, T, cva0 = lib.inner_defaults_cva(w, precision=0, n_b_per_block=nbb, block_paths=64)
    report("T (uneven n_b)", scale_err(npy(T), ref["T"]), 1e-12)
    out = lib.outer_paths(w, precision=0, want_features=False)
    cnt = npy(lib.inner_defaults(w.grid, 1, w.seed, out["Lam"], n_b_per_block=nbb, block_paths=64))
    assert np.array_equal(cnt, ref["cnt"])


def test_single_path_and_single_draw(lib):
    w = wl.plain_fp64().with_(M=1, n_b=1)
    ref = pipeline.simulate(w)
    _, T, cva0 = lib.inner_defaults_cva(w, precision=0)
    report("T (M=1, n_b=1)", scale_err(npy(T), ref["T"]) if ref["T"].any() else
           float(np.max(np.abs(npy(T)))), 1e-12)


def test_scale_workload_sampled_paths(lib):
    """At the full 10-currency / 8-counterparty size and launch shape (M = 2^17), 40 sampled paths
    (both ends, block edges and seeded random ones) match the oracle: features, I, Lambda, MtM,
    the discounted exposures D, and the targets."""
    import torch
    w = wl.cva_at_scale()
    s = lib.Solver(w, precision=1)
    feats, T, cva0 = s.inner_defaults_cva()
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    sample = np.unique(np.concatenate([[0, 1, 63, 64, 4097, 65535, 99999, w.M - 1],
                                       rng.integers(0, w.M, 32)]))
    idx = torch.as_tensor(sample, device="cuda")
    fixed = model.fixed_rates(w)
    o = model.simulate_outer(w, sample)
    mt = model.mtm(w, o, fixed)
    D = model.exposure(w, o, mt)
    F = model.features(w, o)
    Fg = npy(feats[:, :, idx]).astype(np.float64)
    print(f"[cva_at_scale, {sample.size} sampled paths]")
    for f in range(F.shape[1]):
        report(f"feature {f}", scale_err(Fg[:, f], F[:, f]), 1e-5)
    out = lib.outer_paths(w, precision=1, want_features=False, want_mtm=True)
    report("I", scale_err(npy(out["I"][:, idx]), o.I), 1e-5)
    report("Lambda", scale_err(npy(out["Lam"][:, :, idx]), np.transpose(o.Lam, (0, 2, 1))), 1e-5)
    gross = np.maximum(gross_notional(w), 1.0)[None, :, None]
    mg = npy(out["MtM"][:, :, idx]).astype(np.float64)
    report("MtM / gross notional", float(np.max(np.abs(mg - np.transpose(mt, (0, 2, 1))) / gross)), 1e-5)
    dg = npy(out["D"][:, :, idx]).astype(np.float64)
    report("D / gross notional", float(np.max(np.abs(dg - np.transpose(D, (0, 2, 1))) / gross)), 1e-5)
    u = oinner.inner_draws(w, sample)
    js = oinner.default_dates(o.Lam, u)
    xi = oinner.pathwise_loss(o.I, mt, w.market.lgd, js)
    Tref = oinner.targets(xi)
    Tg = npy(T[:, idx]).astype(np.float64)
    report("T sampled", scale_err(Tg, Tref), 1e-5)
    assert np.isfinite(cva0.item()) and cva0.item() > 0


def test_plain_fp32_integrals(lib, case):
    """HSIM_FP32_PLAIN (the baseline with FP32 integrals): the FP32 state and features are those of
    HSIM_FP32 bit for bit (the integrals do not feed back into the state); I and Lambda follow the
    oracle to 1e-4 of their scale (FP32 sums of up to 2500 terms), the exposures D to 1e-4 of the
    gross notional, and every fused output is that of the plain simulation's own stages."""
    w, ref = case
    a = lib.outer_paths(w, precision=lib.HSIM_FP32, want_mtm=True)
    b = lib.outer_paths(w, precision=lib.HSIM_FP32_PLAIN, want_mtm=True)
    m = w.market
    d = 2 * m.n_ccy - 1 + m.n_cpty                     # market factors (not the integral columns)
    assert np.array_equal(npy(a["features"])[:, :d], npy(b["features"])[:, :d])
    assert np.array_equal(npy(a["MtM"]), npy(b["MtM"]))
    eI = scale_err(npy(b["I"]), ref["I"])
    eL = scale_err(npy(b["Lam"]), ref["Lam"])
    g = np.maximum(gross_notional(w), 1.0)[None, :, None]
    eD = float(np.max(np.abs(npy(b["D"]).astype(np.float64) - ref["D"]) / g))
    print(f"  plain FP32 integrals [{w.name}]: I {eI:.2e} (FP64 integrals "
          f"{scale_err(npy(a['I']), ref['I']):.2e}), Lambda {eL:.2e}, D {eD:.2e}", flush=True)
    assert eI <= 1e-4 and eL <= 1e-4 and eD <= 1e-4
    _, T, cva0 = lib.inner_defaults_cva(w, precision=lib.HSIM_FP32_PLAIN)
    cnt = lib.inner_defaults(w.grid, w.market.n_cpty, w.seed, b["Lam"], n_b=w.n_b)
    T2, cva2 = lib.targets_cva(w.grid, w.market.n_cpty, b["I"], b["D"], cnt, n_b=w.n_b)
    assert np.array_equal(npy(T), npy(T2)) and cva0.item() == cva2.item()
