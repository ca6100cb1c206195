"""hsim_targets_cva_noalloc (the allocation-free form of hsim_targets_cva) through the C ABI.

Its results must equal hsim_targets_cva's bit for bit on the same inputs (same kernels, same
fixed-order reduction; only the partials live in the library's static scratch), on two calls in
a row, the second with fewer paths, so that stale partials of the first call would show, in both
precisions and with uneven n_b.  A path count beyond the scratch is refused before any launch.
"""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def npy(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_targets_equal_workspace_targets(lib, precision):
    import torch
    w = wl.small_multi(M=1500, n_b=16)
    out = lib.outer_paths(w, precision=precision, want_features=False)
    C = w.market.n_cpty
    cnt = lib.inner_defaults(w.grid, C, w.seed, out["Lam"], n_b=w.n_b)
    for M in (1500, 333):                       # the second call has fewer paths
        I = out["I"][:, :M].contiguous()
        D = out["D"][:, :, :M].contiguous()
        c = cnt[:, :, :M].contiguous()
        T_ref, cva_ref = lib.targets_cva(w.grid, C, I, D, c, n_b=w.n_b, precision=precision)
        T, cva = lib.targets_cva_noalloc(w.grid, C, I, D, c, n_b=w.n_b, precision=precision)
        torch.cuda.synchronize()
        print(f"  precision {precision} M {M}: cva0 {cva.item():.12g} vs {cva_ref.item():.12g}", flush=True)
        assert torch.equal(T, T_ref)
        assert torch.equal(cva, cva_ref)


def test_noalloc_uneven_nb_equals_workspace(lib):
    import torch
    w = wl.small_multi(M=640, n_b=8)
    levels = np.array([1, 8, 64, 3, 17, 2, 128, 5, 9, 33], dtype=np.int32)
    out = lib.outer_paths(w, precision=1, want_features=False)
    C = w.market.n_cpty
    cnt = lib.inner_defaults(w.grid, C, w.seed, out["Lam"], n_b_per_block=levels, block_paths=64)
    for M, lv in ((640, levels), (192, levels[:3])):
        I = out["I"][:, :M].contiguous()
        D = out["D"][:, :, :M].contiguous()
        c = cnt[:, :, :M].contiguous()
        T_ref, cva_ref = lib.targets_cva(w.grid, C, I, D, c, n_b_per_block=lv, block_paths=64)
        T, cva = lib.targets_cva_noalloc(w.grid, C, I, D, c, n_b_per_block=lv, block_paths=64)
        torch.cuda.synchronize()
        assert torch.equal(T, T_ref) and torch.equal(cva, cva_ref)


def test_noalloc_rejects_paths_beyond_the_scratch(lib):
    import ctypes
    w = wl.small_multi(M=64)
    g = lib.grid_struct(w.grid)
    fake = ctypes.c_void_p(256)                 # never dereferenced: the size check comes first
    rc = lib.lib().hsim_targets_cva_noalloc(ctypes.byref(g), 3, (1 << 24) + 1, 8, None, 64, 1, fake, fake,
                                            fake, fake, fake, lib._stream())
    assert rc == lib.HSIM_ERANGE
    assert b"static scratch" in lib.lib().hsim_last_error()
