"""FP8 storage of sample values, written from its definition (CPU oracle).

TEST INFRASTRUCTURE ONLY: used by the tests to check the library's FP8 packer
and to give the oracle the exact values the FP8 path multiplies.  It shares no
code with the HIP implementation.

The paper computes in FP64; storing the samples of Eq. 3 in FP8 is a
precision option of this implementation, defined as follows.  A value x of
column c is held as x = s_c (q + r):

* s_c is the smallest power of two, clamped to [2^-126, 2^127], for which
  max |x| / s_c <= 448 over the column (the largest finite e4m3 value);
* q is the OCP e4m3 value nearest to x / s_c (ties to the even code;
  beyond 448 the nearest finite value, 448);
* r is the remainder x / s_c - q (exact in FP64) rounded first to FP32 and
  then to BF16, both to nearest with ties to even;
* with two residuals, x = s_c (q + r + t): t is what r leaves of the
  remainder, x / s_c - q - r (exact in FP64), rounded the same way.

Everything here works by enumeration and comparison of exact FP64 values,
not by bit arithmetic on exponents, so that it can be read against the
definition line by line.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np

E4M3_MAX = 448.0


def e4m3_value(code: int) -> float:
    """Value of an OCP e4m3 code byte (sign, 4 exponent bits with bias 7, 3
    mantissa bits; exponent field 0 is subnormal m 2^-9; 0x7F / 0xFF are
    NaN)."""
    sign = -1.0 if code & 0x80 else 1.0
    ef, m = (code >> 3) & 0xF, code & 0x7
    if ef == 0xF and m == 0x7:
        return float("nan")
    if ef == 0:
        return sign * m * 2.0 ** -9
    return sign * (1.0 + m / 8.0) * 2.0 ** (ef - 7)


# the finite non-negative codes 0x00 .. 0x7E in increasing order of value
_POS_CODES = np.arange(0x7F, dtype=np.int64)
_POS_VALUES = np.array([e4m3_value(int(c)) for c in _POS_CODES])
assert np.all(np.diff(_POS_VALUES) > 0)


def e4m3_nearest(a: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Nearest finite e4m3 value to each a >= 0 (ties to the even code) and
    its code.  Values above 448 go to 448."""
    a = np.asarray(a, dtype=np.float64)
    hi = np.clip(np.searchsorted(_POS_VALUES, a, side="left"), 0, len(_POS_VALUES) - 1)
    lo = np.clip(hi - 1, 0, len(_POS_VALUES) - 1)
    dlo = np.abs(a - _POS_VALUES[lo])
    dhi = np.abs(_POS_VALUES[hi] - a)
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (_POS_CODES[hi] % 2 == 0))
    idx = np.where(pick_hi, hi, lo)
    return _POS_VALUES[idx], _POS_CODES[idx]


def column_scales(x: np.ndarray) -> np.ndarray:
    """Smallest power of two s (2^-126 .. 2^127) with max |x[:, c]| / s <= 448,
    per column, found by stepping the exponent."""
    m = np.max(np.abs(x), axis=0) if x.shape[0] else np.zeros(x.shape[1])
    out = np.empty(x.shape[1])
    for c, mc in enumerate(m):
        k = -126
        while k < 127 and mc / 2.0 ** k > E4M3_MAX:
            k += 1
        out[c] = 2.0 ** k
    return out


def _bf16_nearest_bits(f32: np.ndarray) -> np.ndarray:
    """BF16 bit pattern nearest to each FP32 value (ties to even)."""
    bits = f32.view(np.uint32).astype(np.uint64)
    down = bits & 0xFFFF0000                      # toward zero
    up = down + 0x10000                           # next BF16 away from zero
    v = f32.astype(np.float64)
    vd = (down.astype(np.uint32)).view(np.float32).astype(np.float64)
    vu = (up.astype(np.uint32)).view(np.float32).astype(np.float64)
    dd, du = np.abs(v - vd), np.abs(vu - v)
    pick_up = (du < dd) | ((du == dd) & (((up >> 16) & 1) == 0))
    return (np.where(pick_up, up, down) >> 16).astype(np.uint16)


def bf16_value(bits: np.ndarray) -> np.ndarray:
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def fp8_store(x: np.ndarray, residuals: int = 1):
    """Codes [n][c] uint8, residual BF16 bits [n][c] uint16 and scales [c]
    (FP32 values) of x [n][c]; with residuals=2 also the second residual's
    bits, returned after the first: (codes, r bits, t bits, scales)."""
    x = np.asarray(x, dtype=np.float64)
    s = column_scales(x)
    v = x / s                                     # exact: s is a power of two
    qa, code = e4m3_nearest(np.abs(v))
    q = np.where(v < 0, -qa, qa)
    code = np.where((v < 0) & (code != 0), code | 0x80, code).astype(np.uint8)
    rem = v - q                                   # exact
    rbits = _bf16_nearest_bits(rem.astype(np.float32))
    if residuals == 1:
        return code, rbits, s.astype(np.float32)
    rem2 = rem - bf16_value(rbits)                # exact: r is rem to 8 bits
    tbits = _bf16_nearest_bits(rem2.astype(np.float32))
    return code, rbits, tbits, s.astype(np.float32)


def fp8_values(code: np.ndarray, rbits: np.ndarray, scale: np.ndarray, tbits=None) -> np.ndarray:
    """The exact FP64 values s (q + r), or s (q + r + t), that the stored data
    stand for."""
    table = np.array([e4m3_value(c) for c in range(256)])
    v = table[code.astype(np.int64)] + bf16_value(rbits)
    if tbits is not None:
        v = v + bf16_value(tbits)
    return scale.astype(np.float64) * v
