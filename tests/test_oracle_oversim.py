"""Pins of the oversimulation chooser (Section 3.3, Proposition p:heurisN, Heuristic heur:MN)."""
import numpy as np

from oracle import oversim


def test_moments_recover_known_variances():
    """g^{k,l} = A_k + e_{k,l}: R = Var(A), Q = Var(e) (hierarchical sample, exact law)."""
    rng = np.random.default_rng(1)
    M = 400_000
    sR, sQ = 0.7, 1.9
    A = 3.0 + sR * rng.standard_normal(M)
    g1 = A + sQ * rng.standard_normal(M)
    g2 = A + sQ * rng.standard_normal(M)
    R, Q = oversim.r_and_q(oversim.moments(g1[None], g2[None]))
    assert abs(R[0] - sR ** 2) < 0.02 and abs(Q[0] - sQ ** 2) < 0.03


def test_optimum_matches_brute_force_minimiser():
    R, Q, P, Psi = 0.3, 25.0, 497.0, 1e6
    N = np.arange(1, 2000)
    v = np.array([oversim.loss_variance(R, Q, Psi, n, P) for n in N])
    n_star = oversim.optimal_n(Q, R, P)
    assert abs(N[np.argmin(v)] - n_star) <= 1.0
    # the proof's rearranged form: R/Psi ((N - N*)^2 / N + (sqrt(Q/R) + sqrt(P))^2)
    for n in (1.0, 17.0, n_star, 900.0):
        rearranged = R / Psi * ((n - n_star) ** 2 / n + (np.sqrt(Q / R) + np.sqrt(P)) ** 2)
        assert np.isclose(oversim.loss_variance(R, Q, Psi, n, P), rearranged, rtol=1e-12)


def test_cost_ratio_and_heuristic():
    P, c = 497.0, 3.1e-6
    t, tp = c * (P + 1.0), c * (P + 64.0)
    assert np.isclose(oversim.cost_ratio(t, tp, 1.0, 64.0), P, rtol=1e-10)
    N, M = oversim.heuristic([10.0, 20.0, 30.0], P, 1e7)
    assert N == 20.0 and np.isclose(M, 1e7 / 517.0)
    assert oversim.heuristic([0.2, 0.3], P, 1e7)[0] == 1.0      # at least one continuation


def test_pilot_losses_from_common_random_numbers():
    """xi^2 = 2 T(2) - T(1) with T(2) the mean of two continuations whose first is T(1)."""
    rng = np.random.default_rng(2)
    x1, x2 = rng.random((3, 50)), rng.random((3, 50))
    pred = rng.random((3, 50))
    g1, g2 = oversim.losses(x1, 0.5 * (x1 + x2), pred)
    assert np.allclose(g1, (x1 - pred) ** 2) and np.allclose(g2, (x2 - pred) ** 2)
