"""Grouped per-inner-sample regression for one counterparty (Section 3.2 with the default
indicator as X): the alive-group targets and weights of hsim_targets_alive, and the row-weighted
fit of cva_regress_fit, against the FP64 oracle.

Tolerances: targets as the nested targets (FP64 1e-12, FP32 1e-5 scale-relative on paths whose
default counts agree); weights exactly (a ratio of integers rounded once).  The weighted fit
with seeded weights on the three-currency rows is held to the unweighted fits' BF16 bar (2e-2
relative L2 of the predictions, final loss within 1 %).  On the one-counterparty rows (two
inputs, 1000 rows, 8 short epochs) the BF16 and FP64 SGD trajectories part by several per cent
weighted or not, so the alive learner is held to its losses and to the parting of the unweighted
fit of the same rows; an FP32 build of the same kernel source matches the FP64 weighted oracle
to 1e-6 there.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import pipeline
from oracle import regression as org

pytestmark = pytest.mark.gpu


def npy(t):
    return t.detach().cpu().numpy()


def scale_err(got, ref):
    den = max(float(np.max(np.abs(ref))), 1e-300)
    return float(np.max(np.abs(got - ref))) / den


@pytest.fixture(scope="module")
def plain():
    w = wl.plain_fp64().with_(M=1000)                     # ragged last tile
    return w, pipeline.simulate(w, with_alive=True)


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_alive_targets_match_oracle(lib, plain, precision, tol):
    w, ref = plain
    out = lib.outer_paths(w, precision=precision, want_features=False)
    cnt = lib.inner_defaults(w.grid, 1, w.seed, out["Lam"], n_b=w.n_b)
    T, Wt, cva0 = lib.targets_alive(w.grid, out["I"], out["D"], cnt, n_b=w.n_b, precision=precision)
    T, Wt = npy(T).astype(np.float64), npy(Wt).astype(np.float64)
    ok = np.all(npy(cnt) == ref["cnt"], axis=(0, 1))
    assert ok.mean() > 0.99
    err = scale_err(T[:, ok], ref["T_alive"][:, ok])
    print(f"  precision {precision}: T_alive err {err:.3e}, weights exact on {ok.sum()} paths")
    assert err <= tol
    assert np.array_equal(Wt[:, ok], ref["W_alive"][:, ok].astype(np.float32).astype(np.float64))
    _, Tn, cva_n = lib.inner_defaults_cva(w, precision=precision)
    assert cva0.item() == cva_n.item()                  # everyone is alive at t_0
    assert np.array_equal(T[0], npy(Tn)[0].astype(np.float64))


def test_unit_weights_equal_the_unweighted_fit(lib, plain):
    import torch
    w, ref = plain
    X = torch.as_tensor(ref["features"].astype(np.float32), device="cuda")
    Y = torch.as_tensor(ref["T"].astype(np.float32), device="cuda")
    mlp = wl.MLPConfig(hidden=2, width=32, epochs=6, batch=128)
    cfg = lib.mlp_cfg(mlp, X.shape[1], w.M)
    m1, l1, _ = lib.regress_fit(cfg, [10, 30], X, Y, seed=w.seed)
    m2, l2, _ = lib.regress_fit(cfg, [10, 30], X, Y, seed=w.seed, W=torch.ones_like(Y))
    assert torch.equal(m1, m2) and torch.equal(l1, l2)


@pytest.fixture(scope="module")
def multi():
    w = wl.small_multi(M=1024, n_b=16)
    return w, pipeline.simulate(w)


@pytest.mark.parametrize("hidden", [1, 2])
def test_weighted_fit_matches_oracle(lib, multi, hidden):
    """Seeded weights in [0, 2) on the three-currency rows the unweighted fits are checked on."""
    import torch
    w, ref = multi
    dates = [3, 10, 15]
    Wn = np.random.default_rng(1).uniform(0.0, 2.0, ref["T"].shape).astype(np.float32)
    X = torch.as_tensor(ref["features"].astype(np.float32), device="cuda")
    Y = torch.as_tensor(ref["T"].astype(np.float32), device="cuda")
    mlp = wl.MLPConfig(hidden=hidden, width=32, epochs=6, batch=256)
    cfg = lib.mlp_cfg(mlp, X.shape[1], w.M)
    model, loss, _ = lib.regress_fit(cfg, dates, X, Y, seed=w.seed, W=torch.as_tensor(Wn, device="cuda"))
    pred = npy(lib.regress_predict(cfg, dates, X, model)).astype(np.float64)
    fits = org.independent_fits(ref["features"], ref["T"], mlp, w.seed, dates, W=Wn.astype(np.float64))
    for j, i in enumerate(dates):
        p64 = org.predict(fits[i], ref["features"][i].T)
        l2 = np.linalg.norm(pred[j] - p64) / np.linalg.norm(p64)
        print(f"  date {i} hidden {hidden}: l2 {l2:.3e}; loss gpu {npy(loss)[j][-1]:.5f} "
              f"fp64 {fits[i].losses[-1]:.5f}", flush=True)
        assert l2 <= 2e-2
        assert npy(loss)[j][-1] == pytest.approx(fits[i].losses[-1], rel=1e-2)


@pytest.mark.parametrize("hidden", [1, 2])
def test_alive_learner_on_one_counterparty(lib, plain, hidden):
    """The weighted fit of the alive-group targets on the one-counterparty rows: final losses
    agree with the FP64 weighted oracle; the predictions part from it as much as the unweighted
    fit of the same rows does (two inputs, short runs: a BF16-sensitive trajectory)."""
    import torch
    w, ref = plain
    dates = [5, 20, 35]
    X = torch.as_tensor(ref["features"].astype(np.float32), device="cuda")
    Y = torch.as_tensor(ref["T_alive"].astype(np.float32), device="cuda")
    Wt = torch.as_tensor(ref["W_alive"].astype(np.float32), device="cuda")
    mlp = wl.MLPConfig(hidden=hidden, width=32, epochs=8, batch=200)
    cfg = lib.mlp_cfg(mlp, X.shape[1], w.M)
    model, loss, _ = lib.regress_fit(cfg, dates, X, Y, seed=w.seed, W=Wt)
    pred = npy(lib.regress_predict(cfg, dates, X, model)).astype(np.float64)
    fits = org.independent_fits(ref["features"], ref["T_alive"], mlp, w.seed, dates,
                                W=ref["W_alive"].astype(np.float32).astype(np.float64))
    # control: the unweighted fit of the nested targets on the same rows
    Yu = torch.as_tensor(ref["T"].astype(np.float32), device="cuda")
    mu_, _, _ = lib.regress_fit(cfg, dates, X, Yu, seed=w.seed)
    pu = npy(lib.regress_predict(cfg, dates, X, mu_)).astype(np.float64)
    fu = org.independent_fits(ref["features"], ref["T"], mlp, w.seed, dates)
    for j, i in enumerate(dates):
        p64 = org.predict(fits[i], ref["features"][i].T)
        l2 = np.linalg.norm(pred[j] - p64) / np.linalg.norm(p64)
        q64 = org.predict(fu[i], ref["features"][i].T)
        l2u = np.linalg.norm(pu[j] - q64) / np.linalg.norm(q64)
        print(f"  date {i} hidden {hidden}: weighted l2 {l2:.3e} (unweighted control {l2u:.3e}); "
              f"loss gpu {npy(loss)[j][-1]:.5f} fp64 {fits[i].losses[-1]:.5f}", flush=True)
        assert l2 <= max(5e-2, 1.5 * l2u)
        assert npy(loss)[j][-1] == pytest.approx(fits[i].losses[-1], rel=1e-2)
