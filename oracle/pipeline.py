"""Chunked driver of the oracle: outer paths -> prices -> inner draws -> targets.

Arrays are returned in the layouts the library uses, so tests compare them
element by element:  features [n+1, d, P], I [n+1, P], Lam/MtM/D/cnt [n+1, C, P],
T [n+1, P].  P is the number of paths of the requested range.  With ``with_alive`` (one
counterparty) also T_alive / W_alive [n+1, P], the grouped per-inner-sample targets and weights
of ``inner.alive_targets``.
"""
from __future__ import annotations

import numpy as np

from . import inner, model


def simulate(w, path_begin: int = 0, count: int | None = None, n_b: int | None = None,
             chunk: int = 512, market=None, fixed=None, with_moments: bool = False,
             n_b_per_path: np.ndarray | None = None, with_alive: bool = False):
    count = w.M - path_begin if count is None else count
    n_b = w.n_b if n_b is None else n_b
    m = w.market if market is None else market
    fixed = model.fixed_rates(w, m) if fixed is None else fixed
    res = {k: [] for k in ("features", "I", "Lam", "MtM", "D", "cnt", "T", "mu", "var",
                           "T_alive", "W_alive")}
    for c0 in range(path_begin, path_begin + count, chunk):
        paths = np.arange(c0, min(c0 + chunk, path_begin + count))
        outer = model.simulate_outer(w, paths, m)
        mt = model.mtm(w, outer, fixed, m)
        D = model.exposure(w, outer, mt, m)
        res["features"].append(model.features(w, outer))
        res["I"].append(outer.I)
        res["Lam"].append(np.transpose(outer.Lam, (0, 2, 1)))
        res["MtM"].append(np.transpose(mt, (0, 2, 1)))
        res["D"].append(np.transpose(D, (0, 2, 1)))
        if n_b_per_path is None:
            u = inner.inner_draws(w, paths, n_b)
            js = inner.default_dates(outer.Lam, u)
            xi = inner.pathwise_loss(outer.I, mt, m.lgd, js)
            res["cnt"].append(inner.default_counts(js, w.grid.n_dates))
            res["T"].append(inner.targets(xi))
            if with_alive:
                ta, wa = inner.alive_targets(xi, js)
                res["T_alive"].append(ta)
                res["W_alive"].append(wa)
        else:
            # uneven oversimulation: each path uses its own n_b (a prefix of the draws)
            T = np.empty((w.grid.n_dates + 1, paths.shape[0]))
            cnt = np.zeros((w.grid.n_dates + 1, m.n_cpty, paths.shape[0]), dtype=np.int64)
            for lvl in np.unique(n_b_per_path[paths]):
                sel = np.nonzero(n_b_per_path[paths] == lvl)[0]
                u = inner.inner_draws(w, paths[sel], int(lvl))
                Lsel = outer.Lam[:, sel, :]
                js = inner.default_dates(Lsel, u)
                xi = inner.pathwise_loss(outer.I[:, sel], mt[:, sel, :], m.lgd, js)
                T[:, sel] = inner.targets(xi)
                cnt[:, :, sel] = inner.default_counts(js, w.grid.n_dates)
            res["T"].append(T)
            res["cnt"].append(cnt)
        if with_moments:
            mu, var = inner.conditional_moments(outer.I, outer.Lam, mt, m.lgd)
            res["mu"].append(mu)
            res["var"].append(var)
    out = {}
    for k, v in res.items():
        if v:
            out[k] = np.ascontiguousarray(np.concatenate(v, axis=-1))
    out["cva0"] = float(out["T"][0].mean())
    return out
