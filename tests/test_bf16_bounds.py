"""The first-order BF16 error bound used by the GPU one-step test, checked on the CPU.

A NumPy emulation rounds to BF16 (round to nearest even on the upper 16 bits of the FP32 word)
exactly where the library's regression stores BF16 values: standardised inputs, weights,
hidden activations and back-propagated errors; the products are summed in FP64 (tighter than the
GPU's FP32 accumulation, which the bound also covers).  The emulated gradient must lie inside the
bound around the exact FP64 gradient on every element, and a gradient with one element moved
by twice its bound must not (the bound is not vacuous).
"""
import numpy as np
import pytest

import bf16_bounds as bb
from oracle import regression as org


def bf16(x):
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def emulated_gradient(net, X, y, pos):
    B = X.shape[0]
    a = bf16(X)
    acts, pres = [a], []
    for l in range(net.depth):
        z = a @ bf16(net.W[l]).T + net.b[l].astype(np.float32)
        pres.append(z)
        a = bf16(np.maximum(z, 0.0))
        acts.append(a)
    wout = net.W[-1][0].astype(np.float32).astype(np.float64)
    f = a @ wout + np.float32(net.b[-1][0])
    pred = (np.maximum(f, 0.0) if pos else f) + np.float32(net.mu)
    dp = 2.0 * (pred - y) / B
    df = dp * (f > 0.0) if pos else dp
    g_wo = df @ a
    dz = bf16(np.where(a > 0.0, df[:, None] * wout[None, :], 0.0))
    gW, gb = [None] * net.depth, [None] * net.depth
    for l in range(net.depth - 1, -1, -1):
        gW[l] = dz.T @ acts[l]
        gb[l] = dz.sum(axis=0)
        if l > 0:
            dh = dz @ bf16(net.W[l])
            dz = bf16(np.where(acts[l] > 0.0, dh, 0.0))
    out = []
    for l in range(net.depth):
        Wl = np.pad(gW[l], ((0, 0), (0, 32 - gW[l].shape[1]))) if l == 0 else gW[l]
        out += [Wl.reshape(-1), gb[l]]
    out += [g_wo, np.array([df.sum(), dp.sum()])]
    return np.concatenate(out)


@pytest.mark.parametrize("hidden,width,pos", [(1, 32, 0), (2, 32, 1), (3, 64, 0)])
def test_emulated_bf16_gradient_lies_inside_the_bound(hidden, width, pos):
    rng = np.random.default_rng(hidden * 10 + pos)
    M, d = 2048, 9
    X = rng.standard_normal((M, d))
    y = np.log1p(np.exp(X @ rng.standard_normal(d) / 3.0)) + 0.2 * rng.standard_normal(M)
    net = org.init_net(d, hidden, width, seed=hidden)
    net.b = [0.05 * rng.standard_normal(v.size) for v in net.b]
    net.mu = 0.1
    g64, E = bb.gradient_with_bound(net, X, y, pos, 32)
    gW, gb, gmu = org.grads(net, X, y, pos)
    ref = bb.flat_params(org.Net(gW, gb, gmu), 32)
    assert np.allclose(g64, ref, rtol=1e-12, atol=1e-15)             # the exact part is the oracle's
    ge = emulated_gradient(net, X, y, pos)
    ratio = np.abs(ge - g64) / np.maximum(E, 1e-300)
    print(f"  {hidden}x{width} pos={pos}: max |g_bf16 - g64| / bound = {ratio[E > 0].max():.3f}")
    assert np.all(np.abs(ge - g64) <= E)
    assert np.all(ge[E == 0] == g64[E == 0])                           # padded input columns: exact 0
    k = int(np.argmax(E))
    bad = g64.copy()
    bad[k] += 2.0 * E[k]
    assert not np.all(np.abs(bad - g64) <= E)


def test_flat_params_round_trip():
    net = org.init_net(7, 3, 32, seed=4)
    net.mu = 0.25
    flat = bb.flat_params(net, 32)
    back = bb.net_from_flat(flat, 7, 3, 32, 32)
    assert all(np.array_equal(a, b) for a, b in zip(back.W, net.W))
    assert all(np.array_equal(a, b) for a, b in zip(back.b, net.b))
    assert back.mu == net.mu
