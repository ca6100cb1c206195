"""Oversimulation chooser on the GPU: the pilot moments equal the oracle's on the same targets
(FP64 sums of the same FP32 values, 1e-9 relative), and the chooser returns a consistent split."""
import numpy as np
import pytest

import workloads as wl
from oracle import oversim as oos
from oracle import pipeline

pytestmark = pytest.mark.gpu


def test_pilot_moments_match_oracle(lib):
    import torch
    w = wl.small_multi(M=512)
    T1 = pipeline.simulate(w, n_b=1)["T"].astype(np.float32)
    T2 = pipeline.simulate(w, n_b=2)["T"].astype(np.float32)
    pred = (0.5 * T2 + 0.1 * np.random.default_rng(0).random(T2.shape)).astype(np.float32)
    for p in (None, pred):
        ref = oos.moments(*oos.losses(T1, T2, p))
        got = lib.oversim_moments(w.grid, torch.as_tensor(T1, device="cuda"),
                                  torch.as_tensor(T2, device="cuda"),
                                  None if p is None else torch.as_tensor(p, device="cuda")).cpu().numpy()
        scale = np.maximum(np.abs(ref), 1e-300)
        assert np.all(np.abs(got - ref) <= 1e-9 * scale + 1e-300), np.max(np.abs(got - ref) / scale)


def test_chooser_split_is_consistent(lib):
    from paper_2211_17005_amd import oversim
    w = wl.plain_fp64()
    out = oversim.choose(w, Psi=1e8, M_pilot=1 << 16)
    R, Q = out["R"], out["Q"]
    print(f"  P {out['P']:.1f}  N {out['N']:.2f}  M {out['M']:.0f}  "
          f"N*_i range {out['N_dates'].min():.2f}..{out['N_dates'].max():.2f}", flush=True)
    assert out["P"] > 0 and out["N"] >= 1
    assert np.isclose(out["M"] * (out["N"] + out["P"]), 1e8)
    ok = (R > 0) & (Q >= 0)
    assert ok.sum() >= w.grid.n_dates // 2          # dates after the last maturity carry no loss
    assert np.allclose(out["N_dates"], np.sqrt(Q[ok] * out["P"] / R[ok]))
