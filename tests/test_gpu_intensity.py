"""Intensity-based learner targets (Section 4.2, eq. CVAint) through the C ABI, against the FP64
oracle's conditional moments.

The intensity target replaces the inner average of the pathwise loss by its conditional
expectation given the outer path, so it must equal the oracle's mu_i exactly (up to rounding) and
must be the mean, over inner draws, of the nested targets on the same outer paths.

Tolerances: FP64 mode 1e-12 scale-relative (operation order and libm only); FP32 mode 1e-5
scale-relative (the FP32 simulation's own error on D and Lambda).
"""
import numpy as np
import pytest

import workloads as wl
from oracle import inner as oinner
from oracle import model, pipeline

pytestmark = pytest.mark.gpu


def npy(t):
    return t.detach().cpu().numpy()


def scale_err(got, ref):
    den = max(float(np.max(np.abs(ref))), 1e-300)
    return float(np.max(np.abs(got - ref))) / den


def report(name, err, tol):
    print(f"  {name}: err vs FP64 oracle = {err:.3e} (tol {tol:.0e})", flush=True)
    assert err <= tol, (name, err, tol)


CASES = [
    ("plain", lambda: wl.plain_fp64().with_(M=1024)),
    ("small_multi", lambda: wl.small_multi(M=200)),          # ragged last block of paths
    ("tiny", lambda: wl.tiny(M=3)),
    ("single_path", lambda: wl.small_multi(M=1)),
]


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def case(request):
    w = request.param[1]()
    return w, pipeline.simulate(w, with_moments=True)


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_intensity_targets_match_oracle(lib, case, precision, tol):
    w, ref = case
    out = lib.outer_paths(w, precision=precision, want_features=False)
    T, cva0 = lib.targets_intensity(w.grid, w.market.n_cpty, out["I"], out["Lam"], out["D"],
                                    precision=precision)
    T = npy(T).astype(np.float64)
    print(f"[{w.name} M={w.M} precision={precision}]")
    report("T~", scale_err(T, ref["mu"]), tol)
    assert np.all(T[-1] == 0.0)
    cva_ref = float(ref["mu"][0].mean())
    report("CVA_0 (intensity)", abs(cva0.item() - cva_ref) / abs(cva_ref), tol)


def test_intensity_targets_are_the_inner_mean(lib):
    """On the same outer paths, the nested targets with n_b draws scatter around the intensity
    targets with the conditional variance var_i / n_b (eq. CVAint is the conditional mean)."""
    w = wl.small_multi(M=256).with_(n_b=4096)
    ref = pipeline.simulate(w, with_moments=True, n_b=1)
    out = lib.outer_paths(w, precision=0, want_features=False)
    Ti, _ = lib.targets_intensity(w.grid, w.market.n_cpty, out["I"], out["Lam"], out["D"],
                                  precision=0)
    _, Tn, _ = lib.inner_defaults_cva(w, precision=0)
    Ti, Tn = npy(Ti), npy(Tn)
    n = w.grid.n_dates
    # per date, the path sum of T - T~ is a sum of M independent centred terms
    z = (Tn[:n] - Ti[:n]).sum(axis=1) / np.sqrt(ref["var"][:n].sum(axis=1) / w.n_b)
    print(f"  standardised path sums per date: max |z| = {np.abs(z).max():.2f} over {n} dates")
    assert np.all(np.isfinite(z)) and np.abs(z).max() < 5.0
    assert np.all(Ti[n] == 0.0) and np.all(Tn[n] == 0.0)


def test_intensity_targets_scale_workload_sampled_paths(lib):
    """At the 10-currency / 8-counterparty size, M = 2^17, sampled paths match the oracle."""
    import torch
    w = wl.cva_at_scale()
    out = lib.outer_paths(w, precision=1, want_features=False)
    T, cva0 = lib.targets_intensity(w.grid, w.market.n_cpty, out["I"], out["Lam"], out["D"],
                                    precision=1)
    torch.cuda.synchronize()
    sample = np.array([0, 1, 63, 64, 4097, 65535, 99999, w.M - 1])
    o = model.simulate_outer(w, sample)
    mt = model.mtm(w, o, model.fixed_rates(w))
    mu, _ = oinner.conditional_moments(o.I, o.Lam, mt, w.market.lgd)
    Tg = npy(T[:, torch.as_tensor(sample, device="cuda")]).astype(np.float64)
    report("T~ sampled", scale_err(Tg, mu), 1e-5)
    # CVA_0 is the FP64 mean of T~_0 over all paths (reduced before the FP32 rounding of T~)
    assert abs(cva0.item() - float(npy(T[0]).astype(np.float64).mean())) <= 1e-6 * cva0.item()
    _, Tn, cva_nested = lib.inner_defaults_cva(w, precision=1)
    # same outer paths: the nested estimate is the intensity one plus inner noise of order
    # sqrt(var / (n_b M)), far below 1 %
    assert abs(cva_nested.item() - cva0.item()) < 0.01 * cva0.item()
