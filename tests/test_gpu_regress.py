"""Parity of the BF16 MFMA regression (BaseAlg / Backward learning) with the FP64 oracle fit.

Both sides fit the same inputs: the oracle's own features and targets rounded to FP32 (the
library's input type, given to the oracle as FP64), the same initial draw, batch order and Adam
hyper-parameters.

* One Adam step (epochs = 1, batch = M): every gradient element, read back as the Adam moment
  m = (1 - beta1) g, lies within the first-order BF16 rounding bound of the exact FP64 gradient
  (tests/bf16_bounds.py, itself checked against a BF16 emulation on the CPU); v and the stepped
  parameters follow element by element.
* The output-layer refit from a frozen network (lr = 0): the GPU's least-squares weights fit the
  FP64 hidden features to within 1e-3 of the FP64 least-squares minimum loss, and predict within
  the BF16 bar of the oracle's refit.
* Whole fits: predictions within 2e-2 of the FP64 fit both as ||pred - pred64||_2 / ||pred64||_2
  and pointwise as max |pred - pred64| / max |pred64|, on the small cases at width 32 and for
  Backward learning (Algorithm 2) with one hidden layer.  On the oracle's ten-currency case at the
  precision-form shape (29 inputs, 3 x 128 units, batch 8192, 50 epochs, M = 2^17, a team of two
  workgroups per date with loss helpers) exact BF16 arithmetic lands 4-6 % from the FP64 fit (a
  CPU model of the roundings shows it), so the fit is held to the FP64 fit's training loss and
  held-out error, and the kernel at that shape to one exact step and the exact refit.  Wider or deeper networks trained on small
  samples (M <= 8192, a handful of epochs), and the warm-started chain of two hidden layers,
  follow SGD trajectories that BF16 rounding moves apart by more than the bar (a CPU model of the
  kernel's roundings does the same); those shapes are checked by the one-step (also chained
  through Algorithm 2's warm start) and refit tests, and at full size.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import pipeline
from oracle import regression as org

import bf16_bounds as bb

pytestmark = pytest.mark.gpu
TOL = 2e-2


def npy(t):
    return t.detach().cpu().numpy()


def rel_errs(got, ref):
    l2 = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)
    mx = np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300)
    return l2, mx


@pytest.fixture(scope="module")
def data():
    w = wl.small_multi(M=1024, n_b=16)
    r = pipeline.simulate(w)
    return w, r


@pytest.fixture(scope="module")
def data_big():
    w = wl.small_multi(M=8192, n_b=8)
    r = pipeline.simulate(w)
    return w, r


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def fit_both(lib, w, r, mlp, dates, warm, team=0):
    import torch
    F, T = f32(r["features"]), f32(r["T"])
    X = torch.as_tensor(F.astype(np.float32), device="cuda")
    Y = torch.as_tensor(T.astype(np.float32), device="cuda")
    d_in = F.shape[1]
    cfg = lib.mlp_cfg(mlp, d_in, w.M, warm_start=warm, team=team)
    model, loss, _ = lib.regress_fit(cfg, dates, X, Y, seed=w.seed)
    pred = npy(lib.regress_predict(cfg, dates, X, model)).astype(np.float64)
    if warm:
        fits = org.backward_learning(F, T, mlp, w.seed, dates=dates)
    else:
        fits = org.independent_fits(F, T, mlp, w.seed, dates)
    ref = np.stack([org.predict(fits[i], F[i].T) for i in dates])
    loss_ref = np.stack([np.array(fits[i].losses) for i in dates])
    return pred, ref, npy(loss), loss_ref


@pytest.mark.parametrize("width,hidden", [(32, 1), (32, 2)])
def test_independent_fits_match_oracle(lib, data, width, hidden):
    w, r = data
    mlp = wl.MLPConfig(hidden=hidden, width=width, epochs=6, batch=256)
    dates = [3, 10, 15]
    pred, ref, loss, loss_ref = fit_both(lib, w, r, mlp, dates, warm=False)
    for j, i in enumerate(dates):
        l2, mx = rel_errs(pred[j], ref[j])
        print(f"  date {i} width {width}: l2 {l2:.3e} max {mx:.3e}; loss gpu {loss[j][-1]:.5f} "
              f"fp64 {loss_ref[j][-1]:.5f}", flush=True)
        assert l2 <= TOL and mx <= TOL
        assert abs(loss[j][-1] - loss_ref[j][-1]) <= 1e-2 * loss_ref[j][-1]


@pytest.mark.parametrize("team", [1, 2, 3, 8])
def test_team_sizes_match_oracle(lib, data_big, team):
    """A date trained by a team of workgroups (batch gradient summed across them) matches the
    FP64 fit like a single workgroup does; 16 chunks per batch, so team 3 leaves members with
    unequal shares and team 8 two chunks each."""
    w, r = data_big
    mlp = wl.MLPConfig(hidden=2, width=32, epochs=4, batch=1024)
    dates = [3, 10, 15]
    pred, ref, loss, loss_ref = fit_both(lib, w, r, mlp, dates, warm=False, team=team)
    for j, i in enumerate(dates):
        l2, mx = rel_errs(pred[j], ref[j])
        print(f"  team {team} date {i}: l2 {l2:.3e} max {mx:.3e}; loss gpu {loss[j][-1]:.5f} "
              f"fp64 {loss_ref[j][-1]:.5f}", flush=True)
        assert np.all(np.isfinite(loss[j]))
        assert l2 <= TOL and mx <= TOL
        assert abs(loss[j][-1] - loss_ref[j][-1]) <= 1e-2 * loss_ref[j][-1]


def test_team_fit_is_deterministic(lib, data_big):
    import torch
    w, r = data_big
    X = torch.as_tensor(r["features"].astype(np.float32), device="cuda")
    Y = torch.as_tensor(r["T"].astype(np.float32), device="cuda")
    mlp = wl.MLPConfig(hidden=2, width=32, epochs=2, batch=1024)
    cfg = lib.mlp_cfg(mlp, X.shape[1], w.M, team=3)
    m1, l1, _ = lib.regress_fit(cfg, [5, 6, 7], X, Y)
    m2, l2, _ = lib.regress_fit(cfg, [5, 6, 7], X, Y)
    assert torch.equal(m1, m2) and torch.equal(l1, l2)


@pytest.mark.parametrize("big", [False, True])
def test_backward_learning_matches_oracle(lib, data, data_big, big):
    """Algorithm 2 (one date after another, warm-started) with one hidden layer of 32 units; on
    the larger sample every date is trained by a team of workgroups (16 chunks per batch).  With
    two hidden layers the warm-started chain is not a stable comparison: rounding the inputs to
    BF16 alone moves the FP64 chain by 1e-2 to 5e-2 on these samples (a CPU model of the
    kernel's BF16 roundings by 2e-2 to 3e-2); that shape is checked step by step below."""
    w, r = data_big if big else data
    mlp = wl.MLPConfig(hidden=1, width=32, epochs=8 if big else 4, batch=1024 if big else 256)
    dates = [12, 11, 10]
    pred, ref, _, _ = fit_both(lib, w, r, mlp, dates, warm=True)
    for j, i in enumerate(dates):
        l2, mx = rel_errs(pred[j], ref[j])
        print(f"  warm-start date {i}: l2 {l2:.3e} max {mx:.3e}", flush=True)
        assert l2 <= TOL and mx <= TOL


@pytest.mark.parametrize("hidden,width,big", [(2, 32, False), (3, 128, True)])
def test_backward_learning_chain_one_step_elementwise(lib, data, data_big, hidden, width, big):
    """Algorithm 2's warm start, exactly: dates 12 then 11, one Adam step each (epochs = 1,
    batch = M).  Date 11 starts from date 12's result, so its gradient (the Adam moment m / (1 -
    beta1)) must lie within the BF16 bound of the FP64 gradient of date 11's loss at the
    parameters the library stored for date 12."""
    import torch
    w, r = data_big if big else data
    F, T = f32(r["features"]), f32(r["T"])
    M, d = F.shape[2], F.shape[1]
    mlp = wl.MLPConfig(hidden=hidden, width=width, epochs=1, batch=M)
    cfg = lib.mlp_cfg(mlp, d, M, warm_start=True)
    X = torch.as_tensor(F.astype(np.float32), device="cuda")
    Y = torch.as_tensor(T.astype(np.float32), device="cuda")
    model, _, ws = lib.regress_fit(cfg, [12, 11], X, Y, seed=w.seed)
    _, m, _ = (npy(t)[1].astype(np.float64) for t in lib.regress_adam_state(cfg, 2, M, ws))
    npar = m.size
    start = bb.net_from_flat(npy(model)[0][:npar], d, hidden, width, 32)
    Xd, yd = F[11].T, T[11]
    sc = org.scaling(Xd, yd)
    Xs, ys = (Xd - sc.x_mean) / sc.x_std, yd / sc.y_scale
    g64, E = bb.gradient_with_bound(start, Xs, ys, 0, 32)
    g = m / (1.0 - mlp.beta1)
    worst = np.max(np.abs(g - g64) / np.maximum(E, 1e-300))
    print(f"  chained step {hidden}x{width}: max |g - g64| / bound {worst:.3f}", flush=True)
    assert np.all(np.abs(g - g64) <= E + 1e-7 * np.abs(g64))


def test_zero_targets_predict_zero_and_ragged_rows(lib):
    """M = 1000 rows (15 chunks of 64 and a ragged 40) in batches of 200 (batch ends inside
    chunks), an all-zero date that must predict 0; one hidden layer, where the BF16 trajectory
    is stable (a CPU model of the kernel's BF16 roundings moves the FP64 fit by 5e-3)."""
    import torch
    rng = np.random.default_rng(0)
    M = 1000
    X = rng.standard_normal((3, 5, M)).astype(np.float32)
    Y = np.abs(rng.standard_normal((3, M))).astype(np.float32)
    Y[2] = 0.0
    mlp = wl.MLPConfig(hidden=1, width=32, epochs=6, batch=200)
    Xt, Yt = torch.as_tensor(X, device="cuda"), torch.as_tensor(Y, device="cuda")
    cfg = lib.mlp_cfg(mlp, 5, M)
    model, loss, _ = lib.regress_fit(cfg, [1, 2], Xt, Yt, seed=3)
    pred = npy(lib.regress_predict(cfg, [1, 2], Xt, model))
    assert np.all(pred[1] == 0.0)
    fit = org.fit_date(X[1].T.astype(np.float64), Y[1].astype(np.float64), mlp,
                       org.init_net(5, 1, 32, 3), 200)
    ref = org.predict(fit, X[1].T.astype(np.float64))
    l2, mx = rel_errs(pred[0].astype(np.float64), ref)
    print(f"  ragged M={M}: l2 {l2:.3e} max {mx:.3e}")
    assert l2 <= TOL and mx <= TOL


def test_fit_is_deterministic(lib, data):
    import torch
    w, r = data
    X = torch.as_tensor(r["features"].astype(np.float32), device="cuda")
    Y = torch.as_tensor(r["T"].astype(np.float32), device="cuda")
    mlp = wl.MLPConfig(hidden=2, width=32, epochs=2, batch=128)
    cfg = lib.mlp_cfg(mlp, X.shape[1], w.M)
    m1, l1, _ = lib.regress_fit(cfg, [5, 6, 7], X, Y)
    m2, l2, _ = lib.regress_fit(cfg, [5, 6, 7], X, Y)
    assert torch.equal(m1, m2) and torch.equal(l1, l2)


def cfg2_case():
    """The oracle's ten-currency regression case (tests/golden/make_cfg2_regression.py): FP32
    inputs and targets at four dates and the FP64 fits' predictions; written by that script when
    absent (several minutes on the host cores)."""
    import importlib.util
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    spec = importlib.util.spec_from_file_location("make_cfg2_regression",
                                                  os.path.join(here, "golden", "make_cfg2_regression.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    if not os.path.exists(mod.OUT):
        print("  writing the oracle's ten-currency regression case", flush=True)
        mod.main([])
    z = np.load(mod.OUT)
    return {k: z[k] for k in z.files}


@pytest.mark.timeout(1500)
def test_precision_form_fit_on_cva_targets(lib):
    """The benchmarked fit: ten-currency features (29 inputs) and CVA targets of the oracle at
    M = 2^17, 3 x 128 units, batch 8192, 50 epochs, four dates in one launch, a team of two
    workgroups per date with loss helpers.  At this shape the BF16 fit is as good as the FP64 one
    but not the same function: a CPU model of the kernel's BF16 roundings (weights, activations,
    back-propagated errors; FP32 accumulation) lands 3.5e-2 to 5.7e-2 (L2, relative) from the FP64
    fit at these dates, and the GPU as far.  What is asserted is what both estimate: the final
    training loss within 2 % of the FP64 fit's (the rounding model's own final losses lie -0.8 % to
    +0.3 % from it at these dates; the bar is about twice the widest), and the mean squared error
    against the targets of 2^14 held-out paths within 2 % of the FP64 fit's (the equal-accuracy
    bar); the distances between the two predictions are printed.  The kernel's arithmetic at this shape is checked
    exactly by the one-step and refit tests below."""
    import torch
    c = cfg2_case()
    dates = [int(d) for d in c["dates"]]
    n_reg, n_feat, M = c["X"].shape
    w = wl.precision_form(M=M)
    cfg = lib.mlp_cfg(w.mlp, n_feat, M, team=2)
    X = torch.as_tensor(c["X"], device="cuda")
    Y = torch.as_tensor(c["T"], device="cuda")
    rows = list(range(n_reg))
    model, loss, _ = lib.regress_fit(cfg, rows, X, Y, seed=w.seed)
    pred = npy(lib.regress_predict(cfg, rows, X, model)).astype(np.float64)
    Xh = torch.as_tensor(c["X_hold"], device="cuda")
    pred_h = npy(lib.regress_predict(cfg, rows, Xh, model)).astype(np.float64)
    loss = npy(loss).astype(np.float64)
    for j, i in enumerate(dates):
        l2, mx = rel_errs(pred[j], c["pred64"][j])
        Th = c["T_hold"][j].astype(np.float64)
        mse, mse64 = np.mean((pred_h[j] - Th) ** 2), np.mean((c["pred64_hold"][j] - Th) ** 2)
        print(f"  ten-currency date {i}: loss gpu {loss[j][-1]:.6f} fp64 {c['loss64'][j][-1]:.6f}; held-out "
              f"MSE gpu {mse:.6g} fp64 {mse64:.6g} ({mse / mse64 - 1:+.2%}); predictions l2 {l2:.3e} "
              f"max {mx:.3e}", flush=True)
        assert abs(loss[j][-1] - c["loss64"][j][-1]) <= 2e-2 * c["loss64"][j][-1]
        assert abs(mse - mse64) <= 2e-2 * mse64


@pytest.mark.timeout(900)
def test_precision_form_one_step_and_refit_elementwise(lib):
    """At the benchmarked shape and data (29 inputs, 3 x 128, M = 2^17, a team of two): one Adam
    step over all rows matches the FP64 gradient element by element within the BF16 bound, and the
    refit from the frozen initial network reaches the FP64 least-squares loss to 1e-3."""
    import torch
    c = cfg2_case()
    F = c["X"][:1].astype(np.float64)
    T = c["T"][:1].astype(np.float64)
    M, d = F.shape[2], F.shape[1]
    w = wl.precision_form(M=M)
    X = torch.as_tensor(c["X"][:1], device="cuda")
    Y = torch.as_tensor(c["T"][:1], device="cuda")
    Xd, yd = F[0].T, T[0]
    sc = org.scaling(Xd, yd)
    Xs, ys = (Xd - sc.x_mean) / sc.x_std, yd / sc.y_scale
    mlp = wl.MLPConfig(hidden=3, width=128, epochs=1, batch=M)
    cfg = lib.mlp_cfg(mlp, d, M, team=2)
    _, _, ws = lib.regress_fit(cfg, [0], X, Y, seed=w.seed)
    _, m, _ = (npy(t)[0].astype(np.float64) for t in lib.regress_adam_state(cfg, 1, M, ws))
    g64, E = bb.gradient_with_bound(org.init_net(d, 3, 128, w.seed), Xs, ys, 0, 32)
    g = m / (1.0 - mlp.beta1)
    worst = np.max(np.abs(g - g64) / np.maximum(E, 1e-300))
    print(f"  bench shape one step: max |g - g64| / bound {worst:.3f}", flush=True)
    assert np.all(np.abs(g - g64) <= E + 1e-7 * np.abs(g64))
    mlp = wl.MLPConfig(hidden=3, width=128, epochs=2, batch=8192, lr=0.0)
    cfg = lib.mlp_cfg(mlp, d, M, team=2)
    model, _, _ = lib.regress_fit(cfg, [0], X, Y, seed=w.seed)
    npar = bb.flat_params(org.init_net(d, 3, 128, w.seed), 32).size
    got = bb.net_from_flat(npy(model)[0][:npar], d, 3, 128, 32)
    ref = org.init_net(d, 3, 128, w.seed)
    org.refit_output_layer(ref, Xs, ys)
    L64 = org.loss(ref, Xs, ys, 0)
    mix = ref.copy()
    mix.W[-1], mix.b[-1] = got.W[-1], got.b[-1]
    Lgpu = org.loss(mix, Xs, ys, 0)
    print(f"  bench shape refit: loss of the GPU weights {Lgpu:.8f} vs least squares {L64:.8f}", flush=True)
    assert L64 <= Lgpu <= L64 * (1 + 1e-3)


def _one_step_case(lib, F, T, date, hidden, width, seed, tile=0):
    """epochs = 1, batch = M: the fit is one Adam step from the initial draw."""
    import torch
    M, d = F.shape[2], F.shape[1]
    mlp = wl.MLPConfig(hidden=hidden, width=width, epochs=1, batch=M)
    cfg = lib.mlp_cfg(mlp, d, M, team=1, tile=tile)
    X = torch.as_tensor(F.astype(np.float32), device="cuda")
    Y = torch.as_tensor(T.astype(np.float32), device="cuda")
    model, _, ws = lib.regress_fit(cfg, [date], X, Y, seed=seed)
    p, m, v = (npy(t)[0].astype(np.float64) for t in lib.regress_adam_state(cfg, 1, M, ws))
    Xd, yd = F[date].T, T[date]
    sc = org.scaling(Xd, yd)
    Xs, ys = (Xd - sc.x_mean) / sc.x_std, yd / sc.y_scale
    net = org.init_net(d, hidden, width, seed)
    g64, E = bb.gradient_with_bound(net, Xs, ys, 0, 32)
    p0 = bb.flat_params(net, 32).astype(np.float32).astype(np.float64)
    return mlp, p, m, v, g64, E, p0, npy(model)[0].astype(np.float64)


# every wave tiling of the kernels at width 128 (the tilings coincide at width 32)
SHAPES_TILES = [(2, 32, False, 0), (3, 128, True, 0), (3, 128, True, 1), (3, 128, True, 2)]


@pytest.mark.parametrize("hidden,width,big,tile", SHAPES_TILES)
def test_one_adam_step_matches_oracle_elementwise(lib, data, data_big, hidden, width, big, tile):
    w, r = data_big if big else data
    F, T = f32(r["features"]), f32(r["T"])
    mlp, p, m, v, g64, E, p0, rec = _one_step_case(lib, F, T, 10, hidden, width, w.seed, tile)
    b1, b2, lr, eps = mlp.beta1, mlp.beta2, mlp.lr, mlp.eps
    g = m / (1.0 - b1)
    err = np.abs(g - g64)
    worst = np.max(err / np.maximum(E, 1e-300))
    print(f"  one step {hidden}x{width} tiling {tile}: max |g - g64| / bound {worst:.3f}; "
          f"median bound / |g64| {np.median(E / np.maximum(np.abs(g64), 1e-300)):.2e}", flush=True)
    assert np.all(err <= E + 1e-7 * np.abs(g64))                       # m: the gradient
    Ev = (1.0 - b2) * (2.0 * np.abs(g64) * E + E * E)
    assert np.all(np.abs(v - (1.0 - b2) * g64 * g64) <= Ev + 1e-6 * (1.0 - b2) * g64 * g64)
    # the step: -lr g / (|g| + eps) where the sign of g is certain, at most lr where it is not
    sure = np.abs(g64) > E
    step64 = -lr * g64 / (np.abs(g64) + eps)
    slack = lr * eps * E / np.maximum(np.abs(g64) - E + eps, eps) ** 2
    ulp = np.spacing(np.abs(p0).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(p - (p0 + step64))[sure] <= (slack + 4 * ulp + 1e-6 * lr)[sure])
    assert np.all(np.abs(p - p0)[~sure] <= lr * (1 + 1e-5) + 4 * ulp[~sure])
    assert np.array_equal(rec[:p.size], p)                             # the model keeps that step
    print(f"  one step {hidden}x{width}: {sure.mean():.4f} of the parameters with a certain sign",
          flush=True)


@pytest.mark.parametrize("hidden,width,big,tile", SHAPES_TILES)
def test_refit_from_frozen_network_is_least_squares(lib, data, data_big, hidden, width, big, tile):
    """lr = 0 and 2 epochs: the hidden layers keep the initial draw and the refit at the end of
    epoch 1 is the only change (epoch 2 repeats its loss, the first epoch of least loss is kept).
    The GPU's output layer, evaluated in FP64 on the exact hidden features, reaches the FP64
    least-squares minimum to 1e-3 (a ridge or a wrong solve would not), and its predictions
    match the oracle's refit within the BF16 bar."""
    import torch
    w, r = data_big if big else data
    F, T = f32(r["features"]), f32(r["T"])
    M, d = F.shape[2], F.shape[1]
    date = 12
    mlp = wl.MLPConfig(hidden=hidden, width=width, epochs=2, batch=M // 4, lr=0.0)
    cfg = lib.mlp_cfg(mlp, d, M, tile=tile)
    X = torch.as_tensor(F.astype(np.float32), device="cuda")
    Y = torch.as_tensor(T.astype(np.float32), device="cuda")
    model, loss, _ = lib.regress_fit(cfg, [date], X, Y, seed=w.seed)
    pred = npy(lib.regress_predict(cfg, [date], X, model))[0].astype(np.float64)
    npar = bb.flat_params(org.init_net(d, hidden, width, w.seed), 32).size
    got = bb.net_from_flat(npy(model)[0][:npar], d, hidden, width, 32)
    Xd, yd = F[date].T, T[date]
    sc = org.scaling(Xd, yd)
    Xs, ys = (Xd - sc.x_mean) / sc.x_std, yd / sc.y_scale
    ref = org.init_net(d, hidden, width, w.seed)
    for l in range(hidden):                       # the frozen layers: the initial draw, exactly
        assert np.array_equal(got.W[l], ref.W[l].astype(np.float32).astype(np.float64))
        assert np.all(got.b[l] == 0.0)
    org.refit_output_layer(ref, Xs, ys)
    L64 = org.loss(ref, Xs, ys, 0)
    mix = ref.copy()
    mix.W[-1], mix.b[-1] = got.W[-1], got.b[-1]
    Lgpu = org.loss(mix, Xs, ys, 0)
    p64 = org.predict_scaled(ref, Xs, 1) * sc.y_scale
    l2, mx = rel_errs(pred, p64)
    print(f"  refit {hidden}x{width}: loss of the GPU weights {Lgpu:.8f} vs least squares {L64:.8f}; "
          f"pred l2 {l2:.3e} max {mx:.3e}", flush=True)
    assert L64 <= Lgpu <= L64 * (1 + 1e-3)
    assert l2 <= TOL and mx <= TOL


def test_failed_wait_is_reported(lib, data_big):
    """A team barrier that gives up (forced from the host: one poll) fails the call with
    HSIM_ETIMEOUT instead of returning a partial fit; the default limit restores normal fits."""
    import torch
    w, r = data_big
    X = torch.as_tensor(r["features"].astype(np.float32), device="cuda")
    Y = torch.as_tensor(r["T"].astype(np.float32), device="cuda")
    mlp = wl.MLPConfig(hidden=2, width=32, epochs=2, batch=1024)
    cfg = lib.mlp_cfg(mlp, X.shape[1], w.M, team=2)
    lib.set_wait_limit(1)
    try:
        with pytest.raises(lib.HsimError) as ei:
            lib.regress_fit(cfg, [5, 6, 7], X, Y)
        assert ei.value.code == lib.HSIM_ETIMEOUT
    finally:
        lib.set_wait_limit(0)
    model, loss, _ = lib.regress_fit(cfg, [5, 6, 7], X, Y)
    assert torch.all(torch.isfinite(loss))
