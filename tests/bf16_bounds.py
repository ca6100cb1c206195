"""First-order rounding-error bounds of one BF16 gradient evaluation (test helper).

The library's regression stores inputs, weights, activations and back-propagated errors in BF16
(unit roundoff u = 2^-8) and accumulates every product in FP32.  Running the FP64 forward and
backward passes of a network alongside absolute error bounds, in which every BF16 rounding adds
u |value| and every product of two perturbed factors adds |a| E_b + E_a |b|, bounds the gap
between the GPU's gradient and the exact one to first order.  A ReLU whose pre-activation lies
within its own error bound may switch either way; such a unit contributes its full back-propagated
value to the bound.  FP32 accumulation adds 2^-22 of the summed magnitudes.

Returns, for the full-sample gradient at pos = 0 (or pos = 1), the exact gradient and its bound,
both in the parameter order of the library's model record (W_1 padded to `din_pad` columns).
"""
from __future__ import annotations

import numpy as np

U_BF16 = 2.0 ** -8
U_ACC = 2.0 ** -22


def _bf(x):
    return U_BF16 * np.abs(x)


def gradient_with_bound(net, X, y, pos: int, din_pad: int, w=None):
    """net: oracle.regression.Net on standardised data X [B, d], y [B] (scaled targets)."""
    B = X.shape[0]
    acts, Eacts, pres, Epres = [X], [_bf(X)], [], []
    a, Ea = X, _bf(X)
    for l in range(net.depth):
        W, b = net.W[l], net.b[l]
        z = a @ W.T + b
        Ez = Ea @ np.abs(W).T + np.abs(a) @ _bf(W).T + U_ACC * (np.abs(a) @ np.abs(W).T + np.abs(b))
        a = np.maximum(z, 0.0)
        live = (z > 0.0) | (np.abs(z) <= Ez)
        Ea = np.where(live, Ez, 0.0) + _bf(a)
        pres.append(z)
        Epres.append(Ez)
        acts.append(a)
        Eacts.append(Ea)
    wout, bout = net.W[-1][0], net.b[-1][0]
    f = a @ wout + bout
    Ef = Ea @ np.abs(wout) + U_ACC * (np.abs(a) @ np.abs(wout) + abs(bout))
    pred = (np.maximum(f, 0.0) if pos else f) + net.mu
    ww = np.ones(B) if w is None else w
    dp = 2.0 * ww * (pred - y) / B
    Edp = 2.0 * ww * Ef / B
    if pos:
        on = f > 0.0
        amb = np.abs(f) <= Ef
        df = np.where(on, dp, 0.0)
        Edf = np.where(on | amb, Edp, 0.0) + np.where(amb, np.abs(dp), 0.0)
    else:
        df, Edf = dp, Edp
    g_mu, E_mu = dp.sum(), Edp.sum() + U_ACC * np.abs(dp).sum()
    g_bo, E_bo = df.sum(), Edf.sum() + U_ACC * np.abs(df).sum()
    g_wo = df @ a
    E_wo = Edf @ np.abs(a) + np.abs(df) @ Ea + U_ACC * (np.abs(df) @ np.abs(a))
    gW, EW, gb, Eb = [None] * net.depth, [None] * net.depth, [None] * net.depth, [None] * net.depth
    da = df[:, None] * wout[None, :]
    Eda = Edf[:, None] * np.abs(wout)[None, :]
    for l in range(net.depth - 1, -1, -1):
        z, Ez = pres[l], Epres[l]
        on = z > 0.0
        amb = np.abs(z) <= Ez
        dz = np.where(on, da, 0.0)
        Edz = np.where(on | amb, Eda, 0.0) + np.where(amb, np.abs(da), 0.0) + _bf(dz)
        ap, Eap = acts[l], Eacts[l]
        gW[l] = dz.T @ ap
        EW[l] = Edz.T @ np.abs(ap) + np.abs(dz).T @ Eap + U_ACC * (np.abs(dz).T @ np.abs(ap))
        gb[l] = dz.sum(axis=0)
        Eb[l] = Edz.sum(axis=0) + U_ACC * np.abs(dz).sum(axis=0)
        W = net.W[l]
        da = dz @ W
        Eda = Edz @ np.abs(W) + np.abs(dz) @ _bf(W)
    g, E = [], []
    for l in range(net.depth):
        gl, El = gW[l], EW[l]
        if l == 0:
            pad = din_pad - gl.shape[1]
            gl = np.pad(gl, ((0, 0), (0, pad)))
            El = np.pad(El, ((0, 0), (0, pad)))
        g += [gl.reshape(-1), gb[l]]
        E += [El.reshape(-1), Eb[l]]
    g += [g_wo, np.array([g_bo, g_mu])]
    E += [E_wo, np.array([E_bo, E_mu])]
    return np.concatenate(g), np.concatenate(E)


def flat_params(net, din_pad: int):
    """The oracle network's parameters in the model record's order (W_1 padded to din_pad)."""
    out = []
    for l in range(net.depth):
        W = net.W[l]
        if l == 0:
            W = np.pad(W, ((0, 0), (0, din_pad - W.shape[1])))
        out += [W.reshape(-1), net.b[l]]
    out += [net.W[-1][0], np.array([net.b[-1][0], net.mu])]
    return np.concatenate(out)


def net_from_flat(flat, d_in: int, hidden: int, width: int, din_pad: int):
    """Inverse of flat_params: an oracle Net from a model record's parameter block."""
    from oracle import regression as org
    W, b, o = [], [], 0
    fan = din_pad
    for l in range(hidden):
        Wl = np.asarray(flat[o:o + width * fan], dtype=np.float64).reshape(width, fan)
        o += width * fan
        W.append(Wl[:, :d_in].copy() if l == 0 else Wl)
        b.append(np.asarray(flat[o:o + width], dtype=np.float64))
        o += width
        fan = width
    W.append(np.asarray(flat[o:o + width], dtype=np.float64)[None, :])
    o += width
    b.append(np.array([float(flat[o])]))
    mu = float(flat[o + 1])
    return org.Net(W, b, mu)
