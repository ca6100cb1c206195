"""Oversimulation chooser on the GPU: the pilot moments equal the oracle's on the same targets
(FP64 sums of the same FP32 values, 1e-9 relative), and the library's chooser equals the oracle's on them."""
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


def test_chooser_matches_oracle_on_the_pilot(lib):
    """The library's chooser on a GPU pilot equals the oracle's Proposition p:heurisN / Heuristic
    heur:MN applied to the same pilot moments and cost ratio; N*_i is defined at the dates before
    the last swap maturity and at none after it (no loss there)."""
    from oracle import oversim as oos
    from paper_2211_17005_amd import oversim
    w = wl.plain_fp64()
    out = oversim.choose(w, Psi=1e8, M_pilot=1 << 16)
    R, Q = oos.r_and_q(out["moments"])
    ok = (R > 0) & (Q >= 0)
    Ns = oos.optimal_n(Q[ok], R[ok], out["P"])
    N, M = oos.heuristic(Ns, out["P"], 1e8)
    print(f"  P {out['P']:.1f}  N {out['N']:.2f}  M {out['M']:.0f}  "
          f"N*_i range {np.nanmin(out['N_dates']):.2f}..{np.nanmax(out['N_dates']):.2f}", flush=True)
    assert out["P"] > 0 and out["N"] >= 1
    assert np.allclose(out["R"], R, rtol=1e-13, atol=0) and np.allclose(out["Q"], Q, rtol=1e-13, atol=0)
    assert np.array_equal(np.isfinite(out["N_dates"]), ok)
    assert np.allclose(out["N_dates"][ok], Ns, rtol=1e-13)
    assert np.isclose(out["N"], N, rtol=1e-13) and np.isclose(out["M"], M, rtol=1e-13)
    step = w.grid.horizon / w.grid.n_dates
    last = int(np.rint(np.max(w.portfolio.maturity) / step))      # pricing date of the last maturity
    assert np.all(ok[1:last - 2])      # the last dates before maturity carry almost no loss: their R can
    assert not np.any(ok[last:])       # fall below 0 by sampling error, which rules them out
