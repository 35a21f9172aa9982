"""Counter-based normal numbers and the planted serving-job tensors.

Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11): a 128-bit counter and a 64-bit key; ten rounds, each
multiplying counter words 0 and 2 by 0xD2511F53 and 0xCD9E8D57, exchanging
the high and low halves of the products with words 1 and 3 and the key, and
bumping the key by the Weyl constants 0x9E3779B9 / 0xBB67AE85 between rounds.

Normals (Box-Muller): normal number e of stream ``sid`` under key ``seed`` is
taken from pair p = e // 2, drawn at counter (p mod 2^32, p >> 32, sid, 0);
words (0,1) and (2,3) give 53-bit uniforms u, v = (m + 0.5) 2^-53; element 2p
is sqrt(-2 ln u) cos(2 pi v), element 2p+1 uses sin.

Planted job (the paper's synthetic recipe, Sec. 4): true cores N(0,1) from
streams 0x100 + k, X_true = TR(cores) rounded to the storage type, then
X = X_true + eta (||X_true|| / ||E||) E with E from stream 0 (element = linear
index of X, first index fastest), added in FP64 and rounded again; initial
cores N(0,1) from streams 0x200 + k.  The device generator of the serving
library follows the same definition; this module is its host counterpart for
tests.  Nothing here runs an ALS step.
"""
from __future__ import annotations

import math

import numpy as np

from .synth import _ring, planted_tensor

SID_NOISE = 0
SID_TRUE = 0x100
SID_INIT = 0x200

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox4x32-10 of counters ``ctr`` (array (..., 4) of uint32 values) under
    ``key`` (two uint32 values).  Returns uint64 arrays holding 32-bit words."""
    c = [np.asarray(ctr[..., w], dtype=np.uint64) & _MASK for w in range(4)]
    k0 = np.uint64(int(key[0]) & 0xFFFFFFFF)
    k1 = np.uint64(int(key[1]) & 0xFFFFFFFF)
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c = [(hi1 ^ c[1] ^ k0) & _MASK, lo1, (hi0 ^ c[3] ^ k1) & _MASK, lo0]
    return np.stack(c, axis=-1)


def philox_normals(seed: int, sid: int, n: int, start: int = 0) -> np.ndarray:
    """Normal numbers start..start+n-1 of stream ``sid`` under key ``seed``."""
    e = np.arange(start, start + n, dtype=np.uint64)
    p = e >> np.uint64(1)
    ctr = np.stack([p & _MASK, p >> np.uint64(32), np.full_like(p, sid), np.zeros_like(p)], axis=-1)
    seed = int(seed) & ((1 << 64) - 1)
    w = philox4x32_10(ctr, (seed & 0xFFFFFFFF, seed >> 32))
    a = ((w[..., 1] << np.uint64(32)) | w[..., 0]) >> np.uint64(11)
    b = ((w[..., 3] << np.uint64(32)) | w[..., 2]) >> np.uint64(11)
    u = (a.astype(np.float64) + 0.5) * 2.0 ** -53
    v = (b.astype(np.float64) + 0.5) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u))
    t = 6.283185307179586 * v
    return np.where((e & np.uint64(1)) == 1, r * np.sin(t), r * np.cos(t))


def philox_cores(dims, ranks, seed: int, base_sid: int):
    """Cores R_k x I_k x R_{k+1} (Fortran order) of normals from streams base_sid + k."""
    rr = _ring(ranks)
    out = []
    for k, I in enumerate(dims):
        n = rr[k] * int(I) * rr[k + 1]
        out.append(np.asfortranarray(philox_normals(seed, base_sid + k, n).reshape((rr[k], int(I), rr[k + 1]),
                                                                                  order="F")))
    return out


def planted_job(dims, ranks, seed: int, eta: float, dtype=np.float32):
    """(X, true cores, initial cores) of a serving job, as the device generator
    defines them."""
    true = philox_cores(dims, ranks, seed, SID_TRUE)
    init = philox_cores(dims, ranks, seed, SID_INIT)
    xt = planted_tensor(true)
    X = xt.astype(dtype)
    if eta != 0.0:
        flat = philox_normals(seed, SID_NOISE, int(math.prod(dims)))
        E = flat.reshape(tuple(int(d) for d in dims), order="F")
        scale = eta * np.sqrt(np.sum(xt * xt)) / np.sqrt(np.sum(flat * flat))
        X = (X.astype(np.float64) + scale * E).astype(dtype)
    return np.asfortranarray(X), true, init
