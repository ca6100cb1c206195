"""Choice of the oversimulation factor (Section 3.3): Proposition p:heurisN, Heuristic heur:MN
and the cost-ratio identity l:ratio, in FP64 NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

With the loss estimator (1/(M N)) sum_k sum_l g^{k,l} of a date, the outer paths k independent
and the N inner continuations of a path conditionally independent given it:
  R = Cov(g^{k,1}, g^{k,2}) = Var(E[g | outer path]),
  Q = E[Var(g | outer path)] = Var(g) - R,
estimated from a pilot with two inner continuations per outer path:
  R = E[g g'] - E[g]^2,   Q = E[g^2] - E[g g']   (the moments of the proof).
Under the budget M (N + P) = Psi the variance is minimised at N* = sqrt(Q P / R) (e:optom);
Heuristic heur:MN takes for N the average of the per-date N*_i and M = Psi / (N + P); P, the
cost of one outer path in units of one inner continuation, follows from two timings at the same
M (l:ratio): t / t' = (P + N) / (P + N').

Reading: for the targets regressed here the pointwise loss of a date is g = (xi - phi(x))^2 with
xi one inner continuation's pathwise loss and phi the current prediction (0 before training).
With common random numbers the pilot's two continuations come from the n_b = 1 and n_b = 2
targets of the same seed: xi^1 = T(1), xi^2 = 2 T(2) - T(1).
"""
from __future__ import annotations

import numpy as np


def losses(T1: np.ndarray, T2: np.ndarray, pred=None):
    """Pointwise losses of the two pilot continuations, [dates][M] each."""
    xi1 = np.asarray(T1, dtype=np.float64)
    xi2 = 2.0 * np.asarray(T2, dtype=np.float64) - xi1
    phi = 0.0 if pred is None else np.asarray(pred, dtype=np.float64)
    return (xi1 - phi) ** 2, (xi2 - phi) ** 2


def moments(g1: np.ndarray, g2: np.ndarray) -> np.ndarray:
    """Per date (rows of g1, g2): E[g], E[g^2] (both continuations pooled), E[g g']; [dates][3]."""
    mean_g = 0.5 * (g1.mean(axis=-1) + g2.mean(axis=-1))
    mean_g2 = 0.5 * ((g1 * g1).mean(axis=-1) + (g2 * g2).mean(axis=-1))
    mean_gg = (g1 * g2).mean(axis=-1)
    return np.stack([mean_g, mean_g2, mean_gg], axis=-1)


def r_and_q(mom: np.ndarray):
    """R and Q of every date from its three pilot moments."""
    mom = np.asarray(mom, dtype=np.float64)
    R = mom[..., 2] - mom[..., 0] ** 2
    Q = mom[..., 1] - mom[..., 2]
    return R, Q


def optimal_n(Q, R, P):
    """e:optom: N* = sqrt(Q P / R)."""
    return np.sqrt(np.asarray(Q) * P / np.asarray(R))


def loss_variance(R: float, Q: float, Psi: float, N: float, P: float) -> float:
    """Variance of the loss estimator with M = Psi / (N + P) outer paths and N continuations:
    Var = (R + Q / N) / M, each outer path contributing R and each continuation Q."""
    M = Psi / (N + P)
    return (R + Q / N) / M


def cost_ratio(t: float, t_prime: float, N: float, N_prime: float) -> float:
    """P from l:ratio, t / t' = (P + N) / (P + N')."""
    return (t_prime * N - t * N_prime) / (t - t_prime)


def heuristic(N_dates, P: float, Psi: float):
    """Heuristic heur:MN: N = mean of the per-date N*_i (at least 1), M = Psi / (N + P)."""
    N = max(1.0, float(np.mean(N_dates)))
    return N, Psi / (N + P)
