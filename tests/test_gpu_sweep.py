"""Oversimulation on the GPU at large M: properties that hold at any size.

Common random numbers make the first n_b' inner draws of every path a prefix of the first
n_b draws, so targets at different n_b are paired path by path.
  * unbiasedness: mean_k (T^k(n_b) - T^k(1)) = 0 within 5 standard errors;
  * variance law (Section 3.3): Var_k T^k_i = R_i + Q_i / n_b, with R_i the variance of the
    conditional mean given the outer path and Q_i the mean conditional variance of one inner
    draw.  Nested prefixes make it testable without estimating R: for a <= b,
    Cov(T(a), T(b)) = R + Q / b, so the increment T(a) - T(512) is uncorrelated with T(512)
    and its variance is Q (1/a - 1/512), the same Q at every a;
  * uneven n_b in one launch equals the uniform launches path by path (bit-exact).
"""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def npy(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def sweep(lib):
    w = wl.plain_fp64().with_(M=1 << 16)
    out = {}
    for n_b in (1, 2, 8, 64, 512):
        _, T, _ = lib.inner_defaults_cva(w.with_(n_b=n_b), precision=0)
        out[n_b] = npy(T).astype(np.float64)
    return w, out


def test_unbiased_against_single_draw(sweep):
    w, T = sweep
    for n_b in (8, 64, 512):
        for i in (0, 10, 25):
            d = T[n_b][i] - T[1][i]
            assert abs(d.mean()) < 5 * d.std() / np.sqrt(d.size), (n_b, i)


def mean_and_se(z):
    """Sample mean of z and its standard error."""
    return z.mean(), z.std() / np.sqrt(z.size)


def test_variance_law_nested_prefixes(sweep):
    """Var T(n_b) = R + Q/n_b (Section 3.3) through the nested-prefix covariances."""
    w, T = sweep
    top = 512
    for i in (0, 10, 25):
        t = T[top][i] - T[top][i].mean()
        q_hat = {}
        for a in (1, 8, 64):
            inc = T[a][i] - T[top][i]
            c, c_se = mean_and_se((inc - inc.mean()) * t)
            assert abs(c) < 5 * c_se, (i, a, c, c_se)
            d = (inc - inc.mean()) ** 2
            v, v_se = mean_and_se(d)
            scale = 1.0 / (1.0 / a - 1.0 / top)
            q_hat[a] = (v * scale, v_se * scale)
            print(f"  date {i} n_b {a}: Cov(T(a)-T(512), T(512)) {c:.3e} +- {c_se:.1e}; "
                  f"Q {q_hat[a][0]:.4e} +- {q_hat[a][1]:.1e}", flush=True)
        q1, s1 = q_hat[1]
        for a in (8, 64):
            qa, sa = q_hat[a]
            assert abs(qa - q1) < 5 * np.hypot(s1, sa), (i, a, qa, q1)
        # the law itself: Var T(b) = R + Q / b with Q from n_b = 1 and R from n_b = 512
        R = np.var(T[top][i]) - q1 / top
        for b in (8, 64):
            v = np.var(T[b][i])
            pred = R + q1 / b
            d = T[b][i] - T[b][i].mean()
            se = np.sqrt(((d ** 4).mean() - d.var() ** 2) / d.size)
            print(f"  date {i} n_b {b}: var {v:.4e} predicted {pred:.4e} (R {R:.3e})", flush=True)
            assert abs(v - pred) < 5 * (se + s1 * (1.0 / b)), (i, b, v, pred)


def test_uneven_launch_equals_uniform_launches(lib):
    w = wl.oversim_sweep(M=1 << 14)
    nbb = w.extra["n_b_per_block"]
    _, T, _ = lib.inner_defaults_cva(w, precision=1, n_b_per_block=nbb, block_paths=64)
    T = npy(T)
    nbp = np.repeat(nbb, 64)[:w.M]
    for lvl in wl.OVERSIM_LEVELS:
        _, Tu, _ = lib.inner_defaults_cva(w.with_(n_b=int(lvl)), precision=1)
        sel = nbp == lvl
        assert np.array_equal(T[:, sel], npy(Tu)[:, sel]), lvl
