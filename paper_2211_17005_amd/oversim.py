"""Choice of the oversimulation factor N and of the number of outer paths M for a budget
(Section 3.3: Proposition p:heurisN, Heuristic heur:MN, cost ratio l:ratio), on the GPU.

1. Pilot: the targets at n_b = 1 and n_b = 2 of one seed (common random numbers make the first
   continuation of the n_b = 2 run the n_b = 1 run), reduced per date by hsim_oversim_moments
   into the moments of the pointwise loss g = (xi - phi)^2 (phi = the given predictions, 0
   before training).
2. Cost ratio: P, the cost of one outer path in units of one inner continuation, from the
   times of two simulations with the same M and n_b = N, N' (hsim_oversim_cost_ratio).
3. hsim_oversim_choose: R_i = Cov(g, g'), Q_i = E[Var(g | outer path)], N*_i = sqrt(Q_i P / R_i)
   at every date with R_i > 0; N = their mean (at least 1); M = Psi / (N + P) for a budget of
   Psi inner-continuation units.
This module only times the runs and passes the numbers to and from the library.
"""
from __future__ import annotations

from . import hsim


def _timed_solve(w, n_b: int, M: int, reps: int) -> float:
    import torch
    s = hsim.Solver(w.with_(n_b=int(n_b)), precision=hsim.HSIM_FP32, M=M)
    s.inner_defaults_cva(want_features=False)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        s.inner_defaults_cva(want_features=False)
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / reps / 1e3


def pilot(w, M: int, pred=None):
    """Pilot moments [n+1][3] of every date from the n_b = 1, 2 pilot on M outer paths (FP32)."""
    T = []
    for n_b in (1, 2):
        s = hsim.Solver(w.with_(n_b=n_b), precision=hsim.HSIM_FP32, M=M)
        s.inner_defaults_cva(want_features=False)
        T.append(s.T.clone())
    return hsim.oversim_moments(w.grid, T[0], T[1], pred).cpu().numpy()


def cost_ratio(w, M: int, n_b=(1, 1024), reps: int = 5) -> float:
    """P from the times of (M, N) and (M, N') (l:ratio).  N' must be large enough for the inner
    draws to change the time measurably (the outer path can cost thousands of draws)."""
    N, Np = n_b
    t, tp = _timed_solve(w, N, M, reps), _timed_solve(w, Np, M, reps)
    if not tp > t * 1.05:
        raise RuntimeError(f"timings {t:.3g} s (n_b={N}) and {tp:.3g} s (n_b={Np}) do not resolve the "
                           "cost ratio: use a larger M or n_b'")
    return hsim.oversim_cost_ratio(t, tp, N, Np)


def choose(w, Psi: float, M_pilot: int = 1 << 16, pred=None, P=None) -> dict:
    """Heuristic heur:MN for workload w and a budget Psi (in units of one inner continuation)."""
    mom = pilot(w, M_pilot, pred)
    if P is None:
        P = cost_ratio(w, M_pilot)
    out = hsim.oversim_choose(mom, P, Psi)
    out.update({"n_b": int(max(1, round(out["N"]))), "P": float(P), "moments": mom})
    return out
