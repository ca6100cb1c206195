"""Adjoint sensitivities of CVA_0 (smoothed estimator) against finite differences.

Bars (the reading of the FP32 forward): per component |g - g_ref| <= 1e-3 max(|g_ref|, 1e-3 ||g_ref||_inf)
  * against the FP64 oracle's central differences with common random numbers on the same paths,
    for one- and three-currency markets and for the ten-currency / eight-counterparty market at
    all 90 inputs (h = 1e-4 relative, the differentiation form's bump; oracle values stored by
    tests/golden/make_adjoint_cfg2.py);
  * against central differences of the library's own FP32 forward at the full 90-parameter size.
"""
import os
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import sensitivities as osn

pytestmark = pytest.mark.gpu


def npy(t):
    return t.detach().cpu().numpy()


def check_grad(name, g, ref, names, rel=1e-3):
    scale = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
    err = np.abs(g - ref) / scale
    worst = int(np.argmax(err))
    print(f"  {name}: max scaled err {err[worst]:.3e} at {names[worst]} (g={g[worst]:.6g}, ref={ref[worst]:.6g})",
          flush=True)
    assert np.all(err <= rel), [(names[i], g[i], ref[i]) for i in np.nonzero(err > rel)[0]]


@pytest.mark.parametrize("ne,nc", [(1, 1), (3, 3)])
def test_adjoint_matches_oracle_fd(lib, ne, nc):
    w = wl.plain_fp64().with_(M=256) if ne == 1 else wl.small_multi(M=256)
    adj = lib.Adjoint(w)
    cva0, grad = adj()
    g = npy(grad)
    paths = np.arange(w.M)
    ref_cva = osn.cva0_smoothed(w, paths)
    print(f"[{w.name}] CVA_0 smoothed gpu {cva0.item():.8g} oracle {ref_cva:.8g}")
    assert abs(cva0.item() - ref_cva) <= 1e-5 * abs(ref_cva)
    ref = osn.fd_gradient(w, paths, h=1e-4)
    check_grad("adjoint vs FP64 FD", g, ref, osn.names(w.market))


def test_adjoint_matches_oracle_fd_ten_currencies(lib):
    """The 90-input shape the bench times, on the first 512 paths of the differentiation form:
    CVA_0 within the FP32 bar of the oracle's, and every gradient component within 1e-3 of the
    oracle's FP64 central difference at h = 1e-4.  Where that difference quotient is itself moved
    by a kink of (MtM)^+ inside the bump (it then differs from the oracle's h = 1e-5 quotient by
    more than half the bar), the h = 1e-5 quotient is the reference; such inputs are printed."""
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import make_adjoint_cfg2 as golden
    cva_ref, names_ref, fds = golden.load()
    w = wl.differentiation_form(M=golden.PATHS)
    assert names_ref == osn.names(w.market)
    adj = lib.Adjoint(w)
    cva0, grad = adj()
    g = npy(grad)
    print(f"  ten currencies: CVA_0 smoothed gpu {cva0.item():.10g} oracle {cva_ref:.10g}", flush=True)
    assert abs(cva0.item() - cva_ref) <= 1e-5 * abs(cva_ref)
    fd4, fd5 = fds[:, 0], fds[:, 1]
    scale = np.maximum(np.abs(fd4), 1e-3 * np.max(np.abs(fd4)))
    kinked = np.abs(fd4 - fd5) > 0.5e-3 * scale
    for i in np.nonzero(kinked)[0]:
        print(f"  {names_ref[i]}: oracle FD h=1e-4 {fd4[i]:.8g} vs h=1e-5 {fd5[i]:.8g} (kink inside the bump)")
    assert kinked.sum() <= 3
    ref = np.where(kinked, fd5, fd4)
    check_grad("adjoint vs FP64 FD (90 inputs)", g, ref, names_ref)


def test_adjoint_matches_gpu_fd_at_scale(lib):
    """Ten currencies, eight counterparties (90 inputs): adjoint vs the library's own CRN FD."""
    import torch
    w = wl.differentiation_form(M=1 << 14)
    adj = lib.Adjoint(w)
    cva0, grad = adj()
    g = npy(grad).copy()
    base = lib.pack_params(w.market)
    names = osn.names(w.market)
    ref = np.zeros_like(g)
    for k in range(base.size):
        h = 1e-3 * abs(base[k]) if base[k] != 0 else 1e-4
        up, dn = base.copy(), base.copy()
        up[k] += h
        dn[k] -= h
        cu = adj(lib.unpack_params(w.market, up))[0].item()
        cd = adj(lib.unpack_params(w.market, dn))[0].item()
        ref[k] = (cu - cd) / (2 * h)
    torch.cuda.synchronize()
    check_grad("adjoint vs GPU CRN FD (90 inputs)", g, ref, names, rel=5e-3)


def test_autograd_function(lib):
    import torch
    w = wl.small_multi(M=128)
    adj = lib.Adjoint(w)
    CVA = lib.cva_function()
    p = torch.tensor(lib.pack_params(w.market), dtype=torch.float64, requires_grad=True)
    v = CVA.apply(p, adj)
    v.backward()
    _, grad = adj()
    assert np.allclose(p.grad.numpy(), npy(grad))


@pytest.mark.parametrize("name", ["small_multi", "cva_at_scale"])
def test_adjoint_from_forward_outputs_equals_own_forward(lib, name):
    """cva_adjoint_forward on the first M paths of a 2M-path simulation (features with the extra
    columns of the 29-input mode) gives cva_adjoint's results bit for bit."""
    import torch
    w = wl.small_multi(M=512) if name == "small_multi" else wl.cva_at_scale(M=1 << 12)
    adj = lib.Adjoint(w)
    cva0, grad = adj()
    c_ref, g_ref = cva0.clone(), grad.clone()
    s = lib.Solver(w.with_(M=2 * w.M), precision=lib.HSIM_FP32)
    n1, C = w.grid.n_dates + 1, w.market.n_cpty
    feats = torch.empty((n1, s.d, 2 * w.M), dtype=torch.float32, device="cuda")
    I = torch.empty((n1, 2 * w.M), dtype=torch.float64, device="cuda")
    Lam = torch.empty((n1, C, 2 * w.M), dtype=torch.float64, device="cuda")
    D = torch.empty((n1, C, 2 * w.M), dtype=torch.float32, device="cuda")
    lib.check(lib.lib().hsim_outer_paths(lib.ctypes.byref(s.km.struct), lib.ctypes.byref(s.kp.struct),
                                         lib.ctypes.byref(s.g), w.seed, 0, 2 * w.M, lib.HSIM_FP32, s.fm,
                                         lib._dptr(feats), lib._dptr(I), lib._dptr(Lam), lib._dptr(D),
                                         None, lib._stream()))
    cva0, grad = adj.from_forward(feats, I, Lam, D)
    print(f"  {name}: CVA_0 {cva0.item():.10g} vs {c_ref.item():.10g}", flush=True)
    assert torch.equal(cva0, c_ref) and torch.equal(grad, g_ref)
    # the same states kept by the one-launch simulation of the 2M paths (the bench's route)
    fs = lib.FusedSolver(w.with_(M=2 * w.M), precision=lib.HSIM_FP32)
    I.fill_(float("nan")); Lam.fill_(float("nan")); D.fill_(float("nan"))
    f2, _, _ = fs.run_keep(w.M, I, Lam, D)
    cva0, grad = adj.from_forward(f2, I, Lam, D)
    assert torch.equal(cva0, c_ref) and torch.equal(grad, g_ref)
