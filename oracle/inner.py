"""Inner (oversimulated) default draws, pathwise CVA loss and targets (FP64 oracle).

Default rule (Appendix B, e:tau): counterparty c has defaulted by t iff
int_0^t gamma^c >= eps^c with eps^c standard exponential; defaults are checked at
pricing dates only (Remark rem:finecoarse), so the default date index is
j* = min{ j >= 1 : Lambda^c_j >= eps^c }  (none if the set is empty), with
eps = -log(u) for the inner uniform u.

Pathwise loss (Section 4.2, eq:CVA_portfolio), read with the sum over j = i..n-1
(the horizon is the last pricing date) and with the loss-given-default factor:
    xi_i = sum_c sum_{j=i}^{n-1} (beta_{j+1} / beta_i) LGD_c (MtM^c_{j+1})^+ 1{j < tau_c <= j+1}.
It is computed by the backward recursion
    xi_n = 0,  xi_i = (beta_{i+1}/beta_i) (xi_{i+1} + sum_c LGD_c (MtM^c_{i+1})^+ 1{j*_c = i+1}).

Hierarchical simulation (Section 3.2): each outer path k carries n_b conditionally
independent inner draws l.  The target regressed at date i is the inner average
    T^k_i = (1/n_b) sum_l xi^{k,l}_i,
which is an unbiased estimate of E[xi_i | outer path k]; CVA_0 = mean_k T^k_0.
"""
from __future__ import annotations

import numpy as np

from . import philox


def default_dates(Lam: np.ndarray, u: np.ndarray) -> np.ndarray:
    """j*[P, n_b, C] from Lambda[n+1, P, C] and uniforms u[P, n_b, C]; n+1 means no default."""
    n = Lam.shape[0] - 1
    eps = -np.log(u)
    jstar = np.full(u.shape, n + 1, dtype=np.int64)
    for j in range(n, 0, -1):                       # smallest j wins
        hit = Lam[j][:, None, :] >= eps
        jstar = np.where(hit, j, jstar)
    return jstar


def pathwise_loss(I: np.ndarray, mtm_c: np.ndarray, lgd: np.ndarray,
                  jstar: np.ndarray) -> np.ndarray:
    """xi[n+1, P, n_b] by the backward recursion above."""
    n = I.shape[0] - 1
    P, n_b, _ = jstar.shape
    beta = np.exp(-I)
    xi = np.zeros((n + 1, P, n_b))
    for i in range(n - 1, -1, -1):
        loss_next = np.zeros((P, n_b))
        pos = np.maximum(mtm_c[i + 1], 0.0)            # [P, C]
        for c in range(jstar.shape[2]):
            loss_next += lgd[c] * pos[:, c][:, None] * (jstar[:, :, c] == i + 1)
        xi[i] = (beta[i + 1] / beta[i])[:, None] * (xi[i + 1] + loss_next)
    return xi


def targets(xi: np.ndarray) -> np.ndarray:
    """T[n+1, P] = inner average of the pathwise loss."""
    return xi.mean(axis=2)


def alive_targets(xi: np.ndarray, jstar: np.ndarray):
    """Grouped form of the per-inner-sample regression for one counterparty (Section 3.2).

    The paper regresses xi^{k,l}_i on (X^{k,l}_i, Y^k_i) over all (path, draw) samples, with X the
    default indicator 1{tau <= t_i}.  With one counterparty the samples of path k split into the
    dead group (X = 1), whose xi_i is identically 0 (no default remains to be paid), and the alive
    group (X = 0, A^k_i = #{l : j*_l > i} samples); over the alive group
        sum_l (phi - xi^{k,l}_i)^2 = A^k_i (phi - mean_alive xi)^2 + const,
    so the regression on the alive branch is the weighted regression of the alive mean on Y with
    weight A^k_i / n_b: it learns the CVA at t_i given survival of the client.
    Returns (target [n+1, P] = mean of xi over the alive draws, 0 where none is alive;
    weight [n+1, P] = A / n_b).  xi [n+1, P, n_b], jstar [P, n_b, 1].
    """
    if jstar.shape[2] != 1:
        raise ValueError("the alive-group form is exact for one counterparty only")
    n = xi.shape[0] - 1
    n_b = xi.shape[2]
    alive = jstar[None, :, :, 0] > np.arange(n + 1)[:, None, None]      # [n+1, P, n_b]
    A = alive.sum(axis=2)
    s = np.where(alive, xi, 0.0).sum(axis=2)
    target = np.where(A > 0, s / np.maximum(A, 1), 0.0)
    return target, A / n_b


def sample_rows(features: np.ndarray, xi: np.ndarray, jstar: np.ndarray):
    """The paper's per-inner-sample regression data (Section 3.2, hierarchical simulation).

    Every (outer path k, inner draw l) is one sample of I = {1..M} x {1..n_b}: its inputs at
    date i are the market state Y^k_i (the path's features) followed by the default indicators
    X^{k,l}_i = (1{tau_c <= t_i})_c, i.e. 1{j*_c <= i}; its label is the pathwise loss
    xi^{k,l}_i.  Samples are stored in the order (l - 1) M + (k - 1), the order whose
    contiguous slices are the paper's minibatches.
    features [n+1, d, P], xi [n+1, P, n_b], jstar [P, n_b, C]  ->
    X [n+1, d + C, n_b P], Y [n+1, n_b P].
    """
    n1, d, P = features.shape
    n_b, C = jstar.shape[1], jstar.shape[2]
    X = np.empty((n1, d + C, n_b * P))
    Y = np.empty((n1, n_b * P))
    for l in range(n_b):
        cols = slice(l * P, (l + 1) * P)
        X[:, :d, cols] = features
        for i in range(n1):
            X[i, d:, cols] = (jstar[:, l, :] <= i).T
        Y[:, cols] = xi[:, :, l]
    return X, Y


def default_counts(jstar: np.ndarray, n: int) -> np.ndarray:
    """cnt[n+1, C, P]: number of inner draws of each path defaulting at date j."""
    P, _, C = jstar.shape
    cnt = np.zeros((n + 1, C, P), dtype=np.int64)
    for j in range(1, n + 1):
        cnt[j] = (jstar == j).sum(axis=1).T
    return cnt


def conditional_moments(I: np.ndarray, Lam: np.ndarray, mtm_c: np.ndarray, lgd: np.ndarray):
    """Exact mean and variance of xi_i given the outer path, for one inner draw.

    Given the outer path, the eps^c are independent Exp(1), so
    P(j*_c = j) = exp(-Lambda^c_{j-1}) - exp(-Lambda^c_j), and counterparties are
    independent: mu_i = sum_c sum_{j>i} a^c_{ij} p^c_j,
    var_i = sum_c [ sum_{j>i} (a^c_{ij})^2 p^c_j - (sum_{j>i} a^c_{ij} p^c_j)^2 ],
    with a^c_{ij} = LGD_c (beta_j / beta_i) (MtM^c_j)^+.
    This is also the smoothed (conditional) CVA estimator differentiated by the
    sensitivities.
    """
    n = I.shape[0] - 1
    beta = np.exp(-I)
    surv = np.exp(-Lam)                                 # [n+1, P, C]
    p = np.zeros_like(surv)
    p[1:] = surv[:-1] - surv[1:]
    D = lgd[None, None, :] * beta[:, :, None] * np.maximum(mtm_c, 0.0)
    mu = np.zeros((n + 1, I.shape[1]))
    var = np.zeros_like(mu)
    for i in range(n + 1):
        a = D[i + 1:] / beta[i][None, :, None]         # [n-i, P, C]
        pj = p[i + 1:]
        m1 = (a * pj).sum(axis=0)                      # [P, C]
        m2 = (a * a * pj).sum(axis=0)
        mu[i] = m1.sum(axis=1)
        var[i] = (m2 - m1 * m1).sum(axis=1)
    return mu, var


def inner_draws(w, paths, n_b=None) -> np.ndarray:
    n_b = w.n_b if n_b is None else n_b
    return philox.inner_uniforms(w.seed, paths, n_b, w.market.n_cpty)
