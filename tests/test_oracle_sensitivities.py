"""Pins of the oracle's finite-difference CVA_0 sensitivities (CPU)."""
import numpy as np

import workloads as wl
from oracle import sensitivities as sn


def foreign_only(M=64):
    """Two currencies, every swap in the foreign one: MtM (hence CVA_0) is linear in chi_0."""
    corr = np.array([[1.0, 0.3, 0.2], [0.3, 1.0, 0.4], [0.2, 0.4, 1.0]])
    mkt = wl.Market(a=np.array([0.1, 0.12]), b=np.array([0.02, 0.025]),
                    sigma_r=np.array([0.01, 0.011]), r0=np.array([0.02, 0.022]),
                    sigma_fx=np.array([0.2]), fx0=np.array([1.25]), corr=corr,
                    kappa=np.array([0.5, 0.4]), theta=np.array([0.02, 0.03]),
                    nu=np.array([0.1, 0.12]), lambda0=np.array([0.02, 0.04]),
                    lgd=np.array([0.6, 0.5]))
    rng = np.random.default_rng(4)
    book = wl.random_book(rng, 12, 1, 2, max_maturity=5)
    book.ccy[:] = 1
    return wl.Workload(name="foreign_only", market=mkt, portfolio=book,
                       grid=wl.Grid(5.0, 10, 5), M=M, n_b=4, seed=1)


def test_parameter_vector_layout():
    w = wl.cva_at_scale(M=64)
    v = sn.pack(w.market)
    assert v.shape == (90,)
    assert len(sn.names(w.market)) == 90
    m2 = sn.unpack(w.market, v)
    for f in sn.FIELDS:
        assert np.array_equal(getattr(m2, f), getattr(w.market, f))
    assert sn.pack(wl.plain_fp64().market).shape == (8,)


def test_fx0_derivative_is_cva_over_fx0():
    """Homogeneity: CVA_0(c chi_0) = c CVA_0(chi_0) for a foreign-only book."""
    w = foreign_only()
    paths = np.arange(w.M)
    cva = sn.cva0_smoothed(w, paths)
    k = sn.names(w.market).index("fx0[0]")
    g = sn.fd_gradient(w, paths, h=1e-4, index=[k])
    assert np.isclose(g[k], cva / w.market.fx0[0], rtol=1e-7)


def test_central_differences_converge():
    """Central differences are second order: h and h/2 agree to O(h^2)."""
    w = foreign_only(M=32)
    paths = np.arange(w.M)
    names = sn.names(w.market)
    idx = [names.index(n) for n in ("r0[0]", "lambda0[1]", "a[1]", "sigma_fx[0]", "nu[0]")]
    g1 = sn.fd_gradient(w, paths, h=1e-3, index=idx)
    g2 = sn.fd_gradient(w, paths, h=5e-4, index=idx)
    for k in idx:
        assert np.isclose(g1[k], g2[k], rtol=1e-4), names[k]


def test_credit_sensitivities_have_the_expected_sign():
    w = foreign_only(M=64)
    paths = np.arange(w.M)
    names = sn.names(w.market)
    idx = [names.index("lambda0[0]"), names.index("theta[1]")]
    g = sn.fd_gradient(w, paths, h=1e-4, index=idx)
    assert g[idx[0]] > 0 and g[idx[1]] > 0
