"""Philox4x32-10 counter-based generator and the uniform/normal transforms (FP64 oracle).

Philox4x32-R is defined in Salmon, Moraes, Dror & Shaw, "Parallel random numbers:
as easy as 1, 2, 3" (SC'11), Section 3: a 128-bit counter and a 64-bit key, R
rounds of two 32x32->64 products with the multipliers below, XOR mixing, and a
Weyl-sequence key schedule.  R = 10 here.

Counter layout (global indices only, never launch geometry):
  outer normals:  (k, s, f >> 2, 0)  path k, global sub-step s, normal index f
  inner defaults: (k, l >> 2, c, 1)  draw l, counterparty c
  network init:   (layer, idx >> 2, date, 2)
  branch normals: (k, s, 16 b + (f >> 2), 3)  continuation b of path k after its branching
                  date (at most 64 normals per sub-step, so f >> 2 < 16)
Key = (seed mod 2^32, seed >> 32).  The word used is ``l & 3`` (``f & 3``).  Keeping
the draw index l in the first counter word makes the first n_b' draws of every
(path, counterparty) a prefix of the first n_b draws, for any n_b >= n_b'.

The paper does not specify a generator; these are the readings documented for
this build.
"""
from __future__ import annotations

import numpy as np

MASK = np.uint64(0xFFFFFFFF)
M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
ROUNDS = 10

TAG_OUTER = 0
TAG_INNER = 1
TAG_INIT = 2
TAG_BRANCH = 3


def key_from_seed(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Return the four 32-bit output words (as uint64 arrays) for the given counters/key."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & MASK for x in (c0, c1, c2, c3))
    k0 = np.uint64(k0) & MASK
    k1 = np.uint64(k1) & MASK
    for _ in range(ROUNDS):
        p0 = M0 * c0                 # exact: both factors < 2^32
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + W0) & MASK
        k1 = (k1 + W1) & MASK
    return c0, c1, c2, c3


def uniform(x):
    """23-bit uniform on the half-offset grid: u = (2*floor(x / 2^9) + 1) * 2^-24.

    Every value is exactly representable in FP32 and FP64, lies in (0, 1), and
    both precisions therefore see bit-identical uniforms.
    """
    m = np.asarray(x, dtype=np.uint64) >> np.uint64(9)
    return (2.0 * m.astype(np.float64) + 1.0) * 2.0 ** -24


def box_muller(ua, ub):
    """Box & Muller (1958): two independent N(0,1) from two uniforms."""
    rad = np.sqrt(-2.0 * np.log(ua))
    ang = 2.0 * np.pi * ub
    return rad * np.cos(ang), rad * np.sin(ang)


def words(seed, c0, c1, c2, c3):
    k0, k1 = key_from_seed(seed)
    return philox4x32_10(c0, c1, c2, c3, k0, k1)


def outer_normals(seed: int, paths: np.ndarray, s: int, n_z: int, branch=None) -> np.ndarray:
    """Normals z[path, f], f < n_z, for global sub-step s.

    Call (k, s, g, 0) gives words (w0..w3); normals 4g, 4g+1 come from (w0, w1)
    and 4g+2, 4g+3 from (w2, w3), cosine branch first.  With ``branch`` (one index
    b >= 0 per path) the call is (k, s, 16 b + g, 3): the normals of continuation b.
    """
    paths = np.asarray(paths, dtype=np.uint64)
    n_calls = (n_z + 3) // 4
    if n_calls > 16:
        raise ValueError("at most 64 normals per sub-step")
    out = np.empty((paths.shape[0], 4 * n_calls))
    for g in range(n_calls):
        if branch is None:
            w0, w1, w2, w3 = words(seed, paths, s, g, TAG_OUTER)
        else:
            c2 = 16 * np.asarray(branch, dtype=np.uint64) + np.uint64(g)
            w0, w1, w2, w3 = words(seed, paths, s, c2, TAG_BRANCH)
        z0, z1 = box_muller(uniform(w0), uniform(w1))
        z2, z3 = box_muller(uniform(w2), uniform(w3))
        out[:, 4 * g + 0] = z0
        out[:, 4 * g + 1] = z1
        out[:, 4 * g + 2] = z2
        out[:, 4 * g + 3] = z3
    return out[:, :n_z]


def inner_uniforms(seed: int, paths: np.ndarray, n_b: int, n_c: int) -> np.ndarray:
    """Uniforms u[path, l, c] for the inner default draws (draw l, counterparty c)."""
    paths = np.asarray(paths, dtype=np.uint64)
    n_calls = (n_b + 3) // 4
    out = np.empty((paths.shape[0], 4 * n_calls, n_c))
    for c in range(n_c):
        for g in range(n_calls):
            ws = words(seed, paths, g, c, TAG_INNER)
            for j in range(4):
                out[:, 4 * g + j, c] = uniform(ws[j])
    return out[:, :n_b, :]


def raw_words(seed: int, c1: int, c2: int, c3: int, k_begin: int, count: int) -> np.ndarray:
    """Words of counters (k, c1, c2, c3), k = k_begin..k_begin+count-1, flattened [count*4]."""
    ks = np.arange(k_begin, k_begin + count, dtype=np.uint64)
    ws = words(seed, ks, c1, c2, c3)
    return np.stack(ws, axis=1).reshape(-1).astype(np.uint32)
