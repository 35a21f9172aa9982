"""Encoders of the two narrow number formats the X contraction may read,
written from the formats' definitions (not from any library's conversion).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

* BF16: the upper 16 bits of an IEEE binary32 (1 sign, 8 exponent, 7 fraction
  bits), rounded to nearest with ties to even; NaN stays NaN.
* FP8 E4M3 (OCP 8-bit floating point, "E4M3"): 1 sign, 4 exponent bits with
  bias 7, 3 fraction bits; exponent field 0 holds the subnormals m/8 * 2^-6;
  no infinities; S.1111.111 is NaN, so the largest finite magnitude is
  1.75 * 2^8 = 448 (S.1111.110).  Rounding to nearest, ties to even.

The library's FP8 shadow stores fp8(float32(x) * s) with one scale per tensor
s = 448 / max|x| (float32 arithmetic), so ``fp8_e4m3_bits`` takes the scaled
float32 values.

Parity status: pinned in tests/test_oracle_pins.py by values fixed by the
format definitions (exact powers of two, the largest finite value, the
smallest subnormal, ties to even at both ends, signed zero) and by the round
trip of every representable value.
"""
from __future__ import annotations

import numpy as np

__all__ = ["bf16_bits", "bf16_value", "fp8_e4m3_bits", "fp8_e4m3_value", "fp8_shadow_scale"]


def bf16_bits(x) -> np.ndarray:
    """BF16 encodings (uint16) of float32 values: round the 32-bit pattern to
    its upper half, nearest, ties to even."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    upper = u >> 16
    lower = u & 0xFFFF
    round_up = (lower > 0x8000) | ((lower == 0x8000) & ((upper & 1) == 1))
    out = (upper + round_up.astype(np.uint64)) & 0xFFFF
    nan = np.isnan(f)
    out[nan] = (upper[nan] | 0x40) & 0xFFFF          # keep a quiet NaN
    return out.astype(np.uint16)


def bf16_value(bits) -> np.ndarray:
    b = np.asarray(bits, dtype=np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def fp8_e4m3_bits(v) -> np.ndarray:
    """E4M3 encodings (uint8) of float32 values inside the finite range."""
    shape = np.shape(v)
    a = np.atleast_1d(np.asarray(v, dtype=np.float32)).astype(np.float64).ravel()   # exact
    sign = (np.signbit(a)).astype(np.uint8) << 7
    m = np.abs(a)
    out = np.zeros(m.shape, dtype=np.uint8)
    nz = m > 0
    e = np.zeros(m.shape, dtype=np.int64)
    e[nz] = np.floor(np.log2(m[nz])).astype(np.int64)
    # log2 of a binary64 near a power of two: fix the exponent exactly
    lo = nz & (m < np.ldexp(1.0, e))
    e[lo] -= 1
    hi = nz & (m >= np.ldexp(1.0, e + 1))
    e[hi] += 1
    sub = nz & (e < -6)
    # subnormals: multiples of 2^-9
    q = np.rint(np.ldexp(m, 9))                         # ties to even
    out[sub] = np.minimum(q[sub], 8).astype(np.uint8)   # 8 * 2^-9 is the smallest normal (field 0x08)
    norm = nz & ~sub
    frac = np.rint(np.ldexp(m, -e) * 8.0) - 8.0         # 0..8, ties to even
    carry = norm & (frac >= 8)
    e2 = e.copy()
    e2[carry] += 1
    frac[carry] = 0
    field = e2 + 7
    if np.any(norm & ((field > 15) | ((field == 15) & (frac > 6)))):
        raise ValueError("value beyond the largest finite E4M3 magnitude (448)")
    out[norm] = ((field[norm] << 3) | frac[norm].astype(np.int64)).astype(np.uint8)
    return (out | sign).astype(np.uint8).reshape(shape)


def fp8_e4m3_value(bits) -> np.ndarray:
    b = np.asarray(bits, dtype=np.uint8).astype(np.int64)
    s = np.where(b & 0x80, -1.0, 1.0)
    E = (b >> 3) & 0xF
    f = b & 0x7
    val = np.where(E == 0, np.ldexp(f / 8.0, -6), np.ldexp(1.0 + f / 8.0, E - 7))
    val = np.where((E == 15) & (f == 7), np.nan, val)
    return s * val


def fp8_shadow_scale(x) -> np.float32:
    """The per-tensor scale 448 / max|x| in float32 (1 for an all-zero tensor)."""
    am = np.float32(np.max(np.abs(np.asarray(x, dtype=np.float32)))) if np.size(x) else np.float32(0)
    return np.float32(448.0) / am if am > 0 else np.float32(1.0)
