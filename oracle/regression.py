"""Positive neural regression of the CVA targets (FP64 oracle).

Search space NN^+ (Section 2.1, e:nnp): an MLP f with h ReLU hidden layers of
width u and a linear output, and the prediction (f(z))^+ + mu.

Training follows BaseAlg (Algorithm 1, Section 2.2) with Adam (Kingma & Ba 2014)
in place of plain SGD, as the paper says it uses in practice, and Backward
learning (Algorithm 2, Section 2.3) across dates with warm starts.

Readings taken where the listing is garbled or silent:
  * one simultaneous backpropagation step updates all layers and mu per batch;
  * pos = 0 until epoch floor(E/2); at the end of that epoch the output layer
    (W^{h+1}, b^{h+1}) is refitted in closed form by least squares on the full
    sample with the hidden layers frozen and mu fixed (pos = 0 loss; the minimum-norm
    solution where the hidden features are rank deficient); then pos = 1;
  * after every epoch the full-sample pos = 1 loss is evaluated and the best
    parameters are kept (the comparison uses pos = 1 in both halves);
  * the prediction uses the best parameters and the output ReLU: (f)^+ + mu;
  * batches are contiguous ranges of the stored sample order, no shuffling;
  * Adam: lr 1e-3, betas (0.9, 0.999), eps 1e-8, fresh moments for every date;
  * weights drawn U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from the Philox init stream,
    biases and mu start at 0;
  * inputs standardised per date (population mean/std, std 0 -> 1); targets
    divided by their root mean square (no shift, so positivity is kept); a date
    whose targets are all 0 is not trained and predicts 0.

Row weights (optional, w >= 0): every loss becomes (1/|rows|) sum w (pred - y)^2 and the
refit solves the weighted least-squares problem.  With the grouped form of the per-inner-sample
regression (``inner.alive_targets``), the weighted loss over outer paths equals the paper's
loss over all (path, draw) samples of the group up to a constant; integer weights equal
duplicated rows.  The scaling statistics stay unweighted (they only fix units).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

from . import philox


@dataclass
class Net:
    W: List[np.ndarray]          # W[l]: [fan_out, fan_in], l = 0..h (last is [1, width])
    b: List[np.ndarray]
    mu: float = 0.0

    def copy(self) -> "Net":
        return Net([w.copy() for w in self.W], [v.copy() for v in self.b], float(self.mu))

    @property
    def depth(self) -> int:
        return len(self.W) - 1


@dataclass
class Scaling:
    x_mean: np.ndarray
    x_std: np.ndarray
    y_scale: float


@dataclass
class FitResult:
    net: Net
    scaling: Scaling
    best_loss: float
    losses: List[float] = field(default_factory=list)
    trained: bool = True


def layer_shapes(d_in: int, hidden: int, width: int):
    shapes = []
    fan_in = d_in
    for _ in range(hidden):
        shapes.append((width, fan_in))
        fan_in = width
    shapes.append((1, fan_in))
    return shapes


def init_net(d_in: int, hidden: int, width: int, seed: int, date_tag: int = 0) -> Net:
    W, b = [], []
    for l, (fo, fi) in enumerate(layer_shapes(d_in, hidden, width)):
        n = fo * fi
        idx = np.arange(n, dtype=np.uint64)
        k0, k1 = philox.key_from_seed(seed)
        ws = philox.philox4x32_10(np.full(n, l, dtype=np.uint64), idx >> np.uint64(2),
                                  np.full(n, date_tag, dtype=np.uint64),
                                  np.full(n, philox.TAG_INIT, dtype=np.uint64), k0, k1)
        word = np.choose((idx & np.uint64(3)).astype(np.int64), ws)
        u = philox.uniform(word)
        W.append(((2.0 * u - 1.0) / np.sqrt(fi)).reshape(fo, fi))
        b.append(np.zeros(fo))
    return Net(W, b, 0.0)


def forward(net: Net, X: np.ndarray):
    """Return (activations a_0..a_h, pre-activations z_0..z_{h-1}, f)."""
    acts, pres = [X], []
    a = X
    for l in range(net.depth):
        z = a @ net.W[l].T + net.b[l]
        pres.append(z)
        a = np.maximum(z, 0.0)
        acts.append(a)
    f = (a @ net.W[-1].T + net.b[-1])[:, 0]
    return acts, pres, f


def predict_scaled(net: Net, X: np.ndarray, pos: int = 1) -> np.ndarray:
    _, _, f = forward(net, X)
    return (np.maximum(f, 0.0) if pos else f) + net.mu


def loss(net: Net, X, y, pos: int, w=None) -> float:
    r = predict_scaled(net, X, pos) - y
    return float(np.mean(r * r if w is None else w * r * r))


def grads(net: Net, X, y, pos: int, w=None):
    """Gradient of the batch loss (1/|batch|) sum w (pred - y)^2 by backpropagation."""
    acts, pres, f = forward(net, X)
    B = X.shape[0]
    pred = (np.maximum(f, 0.0) if pos else f) + net.mu
    dpred = 2.0 * (pred - y) / B
    if w is not None:
        dpred = dpred * w
    df = dpred * (f > 0.0) if pos else dpred
    gW = [None] * len(net.W)
    gb = [None] * len(net.b)
    gmu = float(dpred.sum())
    gW[-1] = df[None, :] @ acts[-1]
    gb[-1] = np.array([df.sum()])
    da = df[:, None] * net.W[-1]                     # [B, width]
    for l in range(net.depth - 1, -1, -1):
        dz = da * (pres[l] > 0.0)
        gW[l] = dz.T @ acts[l]
        gb[l] = dz.sum(axis=0)
        da = dz @ net.W[l]
    return gW, gb, gmu


class Adam:
    def __init__(self, net: Net, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.t = 0
        self.mW = [np.zeros_like(w) for w in net.W]
        self.vW = [np.zeros_like(w) for w in net.W]
        self.mb = [np.zeros_like(v) for v in net.b]
        self.vb = [np.zeros_like(v) for v in net.b]
        self.mmu = 0.0
        self.vmu = 0.0

    def _upd(self, p, g, m, v):
        m *= self.b1
        m += (1 - self.b1) * g
        v *= self.b2
        v += (1 - self.b2) * g * g
        mh = m / (1 - self.b1 ** self.t)
        vh = v / (1 - self.b2 ** self.t)
        p -= self.lr * mh / (np.sqrt(vh) + self.eps)

    def step(self, net: Net, gW, gb, gmu):
        self.t += 1
        for l in range(len(net.W)):
            self._upd(net.W[l], gW[l], self.mW[l], self.vW[l])
            self._upd(net.b[l], gb[l], self.mb[l], self.vb[l])
        self.mmu = self.b1 * self.mmu + (1 - self.b1) * gmu
        self.vmu = self.b2 * self.vmu + (1 - self.b2) * gmu * gmu
        mh = self.mmu / (1 - self.b1 ** self.t)
        vh = self.vmu / (1 - self.b2 ** self.t)
        net.mu -= self.lr * mh / (np.sqrt(vh) + self.eps)


def refit_output_layer(net: Net, X, y, w=None) -> None:
    """Closed-form least squares for (W^{h+1}, b^{h+1}) with frozen hidden layers, mu fixed.

    Algorithm 1 (Section 2.2) refits the output layer in closed form on the whole sample: the
    argmin over (W^{h+1}, b^{h+1}) of the pos = 0 loss (1/M) sum w (H W + b + mu - y)^2, where H
    are the last hidden layer's activations.  The fitted values of a least-squares problem are
    unique; where [H, 1] is rank deficient (a dead ReLU unit is an all-zero column) the weights
    are not, and the minimum-norm solution is taken (numpy's SVD least squares), which gives a
    zero column weight 0.  Weighted rows scale both sides by sqrt(w).
    """
    acts, _, _ = forward(net, X)
    H = np.concatenate([acts[-1], np.ones((X.shape[0], 1))], axis=1)
    r = y - net.mu
    if w is not None:
        s = np.sqrt(w)
        H = H * s[:, None]
        r = r * s
    sol, *_ = np.linalg.lstsq(H, r, rcond=None)
    net.W[-1] = sol[:-1][None, :].copy()
    net.b[-1] = np.array([sol[-1]])


def batches(M: int, batch: int):
    return [(s, min(s + batch, M)) for s in range(0, M, batch)]


def base_alg(net: Net, X, y, epochs: int, batch: int, lr=1e-3, beta1=0.9, beta2=0.999,
             eps=1e-8, w=None) -> FitResult:
    """BaseAlg on standardised data; returns the best parameters found."""
    opt = Adam(net, lr, beta1, beta2, eps)
    pos = 0
    best = net.copy()
    best_loss = np.inf
    hist = []
    for epoch in range(1, epochs + 1):
        for s, e in batches(X.shape[0], batch):
            gW, gb, gmu = grads(net, X[s:e], y[s:e], pos, None if w is None else w[s:e])
            opt.step(net, gW, gb, gmu)
        if epoch == epochs // 2:
            refit_output_layer(net, X, y, w)
            pos = 1
        L = loss(net, X, y, 1, w)
        hist.append(L)
        if L < best_loss:
            best_loss = L
            best = net.copy()
    return FitResult(best, None, best_loss, hist)


def scaling(X: np.ndarray, y: np.ndarray) -> Scaling:
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std = np.where(std > 0.0, std, 1.0)
    ys = float(np.sqrt(np.mean(y * y)))
    return Scaling(mean, std, ys)


def fit_date(X: np.ndarray, y: np.ndarray, cfg, init: Net, batch: int, w=None) -> FitResult:
    """X [M, d] raw features, y [M] raw targets of one date, w [M] row weights or None."""
    sc = scaling(X, y)
    if sc.y_scale == 0.0:
        return FitResult(init.copy(), sc, 0.0, [], trained=False)
    Xs = (X - sc.x_mean) / sc.x_std
    ys = y / sc.y_scale
    res = base_alg(init.copy(), Xs, ys, cfg.epochs, batch, cfg.lr, cfg.beta1, cfg.beta2, cfg.eps, w)
    res.scaling = sc
    return res


def predict(res: FitResult, X: np.ndarray) -> np.ndarray:
    if not res.trained:
        return np.zeros(X.shape[0])
    Xs = (X - res.scaling.x_mean) / res.scaling.x_std
    return predict_scaled(res.net, Xs, 1) * res.scaling.y_scale


def batch_size(cfg, M: int) -> int:
    if cfg.batch is not None:
        return int(cfg.batch)
    return max(1, M // int(cfg.n_batches))


def backward_learning(features: np.ndarray, T: np.ndarray, cfg, seed: int, dates=None, W=None):
    """Algorithm 2: dates from the last to the first, each warm-started from the later one.

    features [n+1, d, M], T [n+1, M].  Returns {date: FitResult}.
    """
    n = T.shape[0] - 1
    dates = list(range(n, 0, -1)) if dates is None else sorted(dates, reverse=True)
    d_in = features.shape[1]
    M = T.shape[1]
    net = init_net(d_in, cfg.hidden, cfg.width, seed)
    out = {}
    for i in dates:
        res = fit_date(features[i].T, T[i], cfg, net, batch_size(cfg, M), None if W is None else W[i])
        out[i] = res
        if res.trained:
            net = res.net.copy()
    return out


def independent_fits(features: np.ndarray, T: np.ndarray, cfg, seed: int, dates, W=None):
    """Batched reading: every date starts from the same initial network."""
    d_in = features.shape[1]
    M = T.shape[1]
    net = init_net(d_in, cfg.hidden, cfg.width, seed)
    return {i: fit_date(features[i].T, T[i], cfg, net, batch_size(cfg, M), None if W is None else W[i])
            for i in dates}
