"""Branched re-simulation (nested and twin Monte Carlo, Sections 3.3 and 4.3) through the C ABI,
against the FP64 oracle.

Tolerances: the continuation samples xi, FP64 mode 1e-12 scale-relative, FP32 mode 1e-5 (the
FP32 simulation's own error, as for the outer paths); the statistics of hsim_branch_errors,
1e-12 relative (FP64 reductions in a different order).
"""
import numpy as np
import pytest

import workloads as wl
from oracle import branch as obr

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
    # name, workload, date, n_branch
    ("plain_date20", lambda: wl.plain_fp64().with_(M=64), 20, 3),
    ("small_multi_ragged", lambda: wl.small_multi(M=37), 7, 4),
    ("tiny_date0", lambda: wl.tiny(M=3), 0, 2),
]


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def case(request):
    _, make, date, B = request.param
    w = make()
    return w, date, B, obr.branch_targets(w, np.arange(w.M), date, B)


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_branch_samples_match_oracle(lib, case, precision, tol):
    w, date, B, ref = case
    xi = npy(lib.branch_cva(w, date, B, precision=precision))
    print(f"[{w.name} date={date} B={B} precision={precision}]")
    report("xi", scale_err(xi, ref), tol)


def test_last_date_and_range_split(lib):
    w = wl.small_multi(M=200)
    xi = npy(lib.branch_cva(w, w.grid.n_dates, 2, precision=0))
    assert np.all(xi == 0.0)
    full = npy(lib.branch_cva(w, 5, 3, precision=1))
    a = npy(lib.branch_cva(w, 5, 3, precision=1, path_begin=0, M=77))
    b = npy(lib.branch_cva(w, 5, 3, precision=1, path_begin=77, M=123))
    assert np.array_equal(np.concatenate([a, b], axis=1), full)


def test_scale_workload_sampled_paths(lib):
    """10 currencies / 8 counterparties, M = 2^17 paths x 2 continuations from t = 5y."""
    import torch
    w = wl.cva_at_scale()
    date = 50
    xi = lib.branch_cva(w, date, 2, precision=1)
    torch.cuda.synchronize()
    sample = np.array([0, 1, 63, 64, 65535, w.M - 1])
    ref = obr.branch_targets(w, sample, date, 2)
    got = npy(xi[:, torch.as_tensor(sample, device="cuda")])
    report("xi sampled", scale_err(got, ref), 1e-5)
    assert np.all(np.isfinite(npy(xi))) and float(xi.min()) >= 0.0


@pytest.mark.parametrize("B", [2, 5])
@pytest.mark.parametrize("phi_kind", ["fp32", "fp64", "none"])
def test_branch_errors_match_oracle(lib, B, phi_kind):
    import torch
    rng = np.random.default_rng(11 + B)
    M = 3000                                           # ragged last block of 256
    cva = rng.lognormal(0.0, 0.7, M)
    xi = cva[None, :] * (1.0 + 0.5 * rng.standard_normal((B, M)))
    phi = cva * (1.0 + 0.1 * rng.standard_normal(M))
    if phi_kind == "fp32":
        phi = phi.astype(np.float32).astype(np.float64)
        phi_t = torch.as_tensor(phi.astype(np.float32), device="cuda")
    elif phi_kind == "fp64":
        phi_t = torch.as_tensor(phi, device="cuda")
    else:
        phi, phi_t = np.zeros(M), None
    got = lib.branch_errors(torch.as_tensor(xi, device="cuda"), phi_t)
    ref = obr.twin_errors(phi, xi)
    for k in obr.STATS:
        err = abs(got[k] - ref[k]) / max(abs(ref[k]), 1e-300)
        assert err <= 1e-12 or (ref[k] == 0.0 and got[k] == 0.0), (k, got[k], ref[k])


def test_twin_validation_of_learned_cva(lib):
    """Section 3.3 on fitted networks (the comparison of Section 4.3's first experiment): the
    learner on the intensity targets has a smaller twin Monte Carlo L^2 error than the learner
    on single-draw default targets; the twin and nested estimators differ by exactly the
    inner-variance term."""
    import torch
    w = wl.plain_fp64().with_(M=8192, n_b=1)
    date = 25
    mlp = wl.MLPConfig(hidden=2, width=32, epochs=30, batch=512)
    train = lib.outer_paths(w, precision=1)
    test = lib.outer_paths(w, precision=1, path_begin=w.M)
    C = w.market.n_cpty
    _, Tn, _ = lib.inner_defaults_cva(w, precision=1)
    Ti, _ = lib.targets_intensity(w.grid, C, train["I"], train["Lam"], train["D"], precision=1)
    X, Xt = train["features"], test["features"]
    cfg = lib.mlp_cfg(mlp, X.shape[1], w.M)
    xi = lib.branch_cva(w, date, 32, precision=1, path_begin=w.M)
    res = {}
    for name, Y in (("defaults_nb1", Tn), ("intensity", Ti)):
        model, _, _ = lib.regress_fit(cfg, [date], X, Y.contiguous(), seed=w.seed)
        phi = lib.regress_predict(cfg, [date], Xt, model)[0].contiguous()
        st = lib.branch_errors(xi, phi)
        st2 = lib.branch_errors(xi[:2].contiguous(), phi)
        res[name] = st
        rel = np.sqrt(max(st["mse_twin"], 0.0) / st["cva_sq"])
        rel2 = np.sqrt(max(st2["mse_twin"], 0.0) / st2["cva_sq"])
        print(f"  {name}: twin relative L2 error {rel:.3f} (B=32), {rel2:.3f} (B=2); "
              f"mean phi {st['phi_mean']:.4e} vs nested CVA {st['cva_mean']:.4e}", flush=True)
        # nested minus twin is the same inner-variance term, whatever phi is
        assert (st["mse_nested"] - st["mse_twin"]) == pytest.approx(
            st["cva_sq_nested"] - st["cva_sq"], rel=1e-9, abs=1e-12 * st["cva_sq"])
    assert res["intensity"]["mse_twin"] < res["defaults_nb1"]["mse_twin"]
    # the intensity learner tracks the nested benchmark closely on average
    assert res["intensity"]["phi_mean"] == pytest.approx(res["intensity"]["cva_mean"], rel=0.05)
