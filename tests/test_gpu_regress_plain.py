"""The FP32 / FP64 regression path (cva_mlp_cfg.dtype = REG_FP32 / REG_FP64) against the FP64
oracle's BaseAlg (Algorithm 1) and Backward learning (Algorithm 2).

FP64 runs the oracle's arithmetic in another summation order, so the whole fit must agree to
1e-6 (relative L2 and max of the predictions, and the loss histories), including the shapes
where BF16 rounding moves the SGD trajectory by several per cent (two inputs, warm-started chains
of two hidden layers) and the first configuration of the benchmark set (one currency, 2 x 32
units, 200 epochs, batch M / 32, Algorithm 2).  One Adam step matches the FP64 gradient element
by element to 1e-9.  FP32 follows FP64 to 5e-3 on those shapes (its rounding is 2^-24 where
BF16's is 2^-9; the errors are printed) except the warm-started chain of three hidden layers,
where FP32 rounding alone moves the third date by 1.3e-2, which is checked in FP64 only.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import pipeline
from oracle import regression as org

import bf16_bounds as bb

pytestmark = pytest.mark.gpu
TOL64 = 1e-6
TOL32 = 5e-3


def npy(t):
    return t.detach().cpu().numpy()


def rel_errs(got, ref):
    l2 = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)
    mx = np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300)
    return l2, mx


@pytest.fixture(scope="module")
def multi():
    w = wl.small_multi(M=1024, n_b=16)
    return w, pipeline.simulate(w)


@pytest.fixture(scope="module")
def plain1():
    w = wl.plain_fp64().with_(M=1000)
    return w, pipeline.simulate(w, with_alive=True)


def fit_both(lib, w, F, T, mlp, dates, warm, dtype, W=None):
    import torch
    R = torch.float64 if dtype == lib.REG_FP64 else torch.float32
    cast = (lambda a: a) if dtype == lib.REG_FP64 else (lambda a: a.astype(np.float32).astype(np.float64))
    F, T = cast(np.asarray(F, np.float64)), cast(np.asarray(T, np.float64))
    W = None if W is None else cast(np.asarray(W, np.float64))
    X = torch.as_tensor(F, dtype=R, device="cuda")
    Y = torch.as_tensor(T, dtype=R, device="cuda")
    Wt = None if W is None else torch.as_tensor(W, dtype=R, device="cuda")
    cfg = lib.mlp_cfg(mlp, F.shape[1], F.shape[2], warm_start=warm, dtype=dtype)
    model, loss, _ = lib.regress_fit(cfg, dates, X, Y, seed=w.seed, W=Wt)
    pred = npy(lib.regress_predict(cfg, dates, X, model)).astype(np.float64)
    if warm:
        fits = org.backward_learning(F, T, mlp, w.seed, dates=dates, W=W)
    else:
        fits = org.independent_fits(F, T, mlp, w.seed, dates, W=W)
    ref = np.stack([org.predict(fits[i], F[i].T) for i in dates])
    loss_ref = np.stack([np.array(fits[i].losses) for i in dates])
    return pred, ref, npy(loss).astype(np.float64), loss_ref


def check(name, pred, ref, loss, loss_ref, dates, tol):
    for j, i in enumerate(dates):
        l2, mx = rel_errs(pred[j], ref[j])
        lerr = np.max(np.abs(loss[j] - loss_ref[j]) / np.abs(loss_ref[j]))
        print(f"  {name} date {i}: l2 {l2:.3e} max {mx:.3e} loss history {lerr:.3e}", flush=True)
        assert l2 <= tol and mx <= tol and lerr <= tol


@pytest.mark.parametrize("dtype,tol,hidden,warm", [(2, TOL64, 2, False), (1, TOL32, 2, False),
                                                   (2, TOL64, 2, True), (1, TOL32, 2, True),
                                                   (2, TOL64, 3, True)])
def test_fits_match_oracle(lib, multi, dtype, tol, hidden, warm):
    w, r = multi
    mlp = wl.MLPConfig(hidden=hidden, width=32, epochs=4, batch=256)
    dates = [12, 11, 10]
    pred, ref, loss, loss_ref = fit_both(lib, w, r["features"], r["T"], mlp, dates, warm, dtype)
    check(f"dtype {dtype} {hidden}x32 warm {warm}", pred, ref, loss, loss_ref, dates, tol)


@pytest.mark.parametrize("dtype,tol", [(2, TOL64), (1, TOL32)])
def test_alive_learner_matches_oracle(lib, plain1, dtype, tol):
    """The weighted fit of the alive-group targets of one counterparty (two inputs), where the
    BF16 kernel's trajectory is not a stable comparison."""
    w, r = plain1
    mlp = wl.MLPConfig(hidden=2, width=32, epochs=8, batch=200)
    dates = [5, 20, 35]
    pred, ref, loss, loss_ref = fit_both(lib, w, r["features"], r["T_alive"], mlp, dates, False, dtype,
                                         W=r["W_alive"])
    check(f"alive dtype {dtype}", pred, ref, loss, loss_ref, dates, tol)


def test_first_configuration_fp64(lib):
    """One currency, one counterparty, 2 x 32 units, 200 Adam epochs in batches of M / 32 on the
    inputs (r, lambda), Algorithm 2 over the last dates, all in FP64."""
    w = wl.plain_fp64()
    r = pipeline.simulate(w)
    dates = [40, 39, 38]
    pred, ref, loss, loss_ref = fit_both(lib, w, r["features"], r["T"], w.mlp, dates, True, lib.REG_FP64)
    check("first configuration", pred, ref, loss, loss_ref, dates, TOL64)


@pytest.mark.parametrize("hidden,width", [(2, 32), (3, 128)])
def test_one_step_fp64_elementwise(lib, multi, hidden, width):
    """epochs = 1, batch = M: m / (1 - beta1) is the full-sample gradient at the initial draw,
    element by element equal to the oracle's FP64 gradient to 1e-9."""
    import torch
    w, r = multi
    F, T = r["features"], r["T"]
    M, d = F.shape[2], F.shape[1]
    date = 10
    mlp = wl.MLPConfig(hidden=hidden, width=width, epochs=1, batch=M)
    cfg = lib.mlp_cfg(mlp, d, M, dtype=lib.REG_FP64)
    X = torch.as_tensor(F, dtype=torch.float64, device="cuda")
    Y = torch.as_tensor(T, dtype=torch.float64, device="cuda")
    _, _, ws = lib.regress_fit(cfg, [date], X, Y, seed=w.seed)
    p, m, _ = (npy(t)[0] for t in lib.regress_adam_state(cfg, 1, M, ws))
    Xd, yd = F[date].T, T[date]
    sc = org.scaling(Xd, yd)
    Xs, ys = (Xd - sc.x_mean) / sc.x_std, yd / sc.y_scale
    net = org.init_net(d, hidden, width, w.seed)
    gW, gb, gmu = org.grads(net, Xs, ys, 0)
    g64 = bb.flat_params(org.Net(gW, gb, gmu), 32)
    g = m / (1.0 - mlp.beta1)
    err = np.max(np.abs(g - g64) / (np.abs(g64) + 1e-6 * np.max(np.abs(g64))))
    print(f"  FP64 one step {hidden}x{width}: max relative gradient error {err:.3e}", flush=True)
    assert err <= 1e-9
    p0 = bb.flat_params(net, 32)
    step = -mlp.lr * g64 / (np.abs(g64) + mlp.eps)
    assert np.allclose(p, p0 + step, rtol=0, atol=1e-12)


@pytest.mark.parametrize("dtype", [1, 2])
def test_zero_date_and_ragged_rows(lib, dtype):
    """M = 1000 rows in batches of 96 (ragged), a date whose targets are all zero predicts 0."""
    import torch
    R = torch.float64 if dtype == 2 else torch.float32
    rng = np.random.default_rng(0)
    M = 1000
    X = rng.standard_normal((3, 5, M))
    Y = np.abs(rng.standard_normal((3, M)))
    Y[2] = 0.0
    if dtype == 1:
        X, Y = X.astype(np.float32).astype(np.float64), Y.astype(np.float32).astype(np.float64)
    mlp = wl.MLPConfig(hidden=2, width=32, epochs=4, batch=96)
    cfg = lib.mlp_cfg(mlp, 5, M, dtype=dtype)
    Xt, Yt = torch.as_tensor(X, dtype=R, device="cuda"), torch.as_tensor(Y, dtype=R, device="cuda")
    model, loss, _ = lib.regress_fit(cfg, [1, 2], Xt, Yt, seed=3)
    pred = npy(lib.regress_predict(cfg, [1, 2], Xt, model)).astype(np.float64)
    assert np.all(pred[1] == 0.0) and np.all(npy(loss)[1] == 0.0)
    fit = org.fit_date(X[1].T, Y[1], mlp, org.init_net(5, 2, 32, 3), 96)
    l2, mx = rel_errs(pred[0], org.predict(fit, X[1].T))
    print(f"  ragged dtype {dtype}: l2 {l2:.3e} max {mx:.3e}", flush=True)
    tol = TOL64 if dtype == 2 else TOL32
    assert l2 <= tol and mx <= tol
