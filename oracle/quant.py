"""Reference storage encoders for the mixed-precision path.

TEST INFRASTRUCTURE ONLY (same rules as the rest of the oracle).

The mixed mode stores A in BF16 or FP8 and forms the Gram with FP32
accumulation, while the problem it solves is the one on the dequantised matrix
X^ (exact in FP64).  These encoders define X^; both follow the formats'
definitions, rounding FP64 values directly (no intermediate FP32) to nearest,
ties to even:

* BF16: 1 sign, 8 exponent (bias 127), 7 fraction bits; subnormal quantum
  2^-133; results beyond the largest finite value become +-inf.  No scale.
* FP8 E4M3 (OCP "fn" variant): 1 sign, 4 exponent (bias 7), 3 fraction bits;
  largest finite 448, subnormal quantum 2^-9, no infinities; rounding
  saturates at +-448.  Row i is stored as q = E4M3(x / s_i) with the FP32 scale
  s_i = fp32(amax_i / 448) (s_i = 1 for an all-zero row), and X^_ik = q_ik s_i.
"""

import numpy as np

BF16_MAX = float(np.ldexp(2.0 - 2.0 ** -7, 127))
E4M3_MAX = 448.0


def _round_to_grid(v, mant_bits, min_exp):
    """Round FP64 values to nearest-even on a grid with `mant_bits` fraction
    bits and minimum normal exponent `min_exp` (subnormals below it)."""
    v = np.asarray(v, dtype=np.float64)
    m, ex = np.frexp(v)                     # v = m 2^ex, 0.5 <= |m| < 1
    e = np.maximum(ex - 1, min_exp)         # floor(log2|v|), clamped to the subnormal range
    e = np.where(v == 0, min_exp, e)
    q = np.ldexp(np.rint(np.ldexp(v, mant_bits - e)), e - mant_bits)
    return q


def bf16_round(x):
    """Nearest BF16 value (as FP64) of each FP64 input."""
    q = _round_to_grid(x, 7, -126)
    return np.where(np.abs(q) > BF16_MAX, np.copysign(np.inf, q), q)


def bf16_bits(x):
    """uint16 BF16 encodings of FP64 inputs."""
    q = bf16_round(x).astype(np.float32)    # exact: BF16 values are FP32 values
    return (q.view(np.uint32) >> 16).astype(np.uint16)


def e4m3_round(x):
    """Nearest E4M3 value (as FP64), saturating at +-448."""
    q = _round_to_grid(x, 3, -6)
    return np.clip(q, -E4M3_MAX, E4M3_MAX)


def e4m3_bits(x):
    """uint8 E4M3 encodings of FP64 inputs (after saturating rounding)."""
    q = e4m3_round(x)
    sign = (np.signbit(q)).astype(np.uint8) << 7
    a = np.abs(q)
    out = np.zeros(a.shape, dtype=np.uint8)
    sub = a < 2.0 ** -6
    out[sub] = np.rint(a[sub] / 2.0 ** -9).astype(np.uint8)           # E = 0, M = a / 2^-9
    nz = ~sub
    m, ex = np.frexp(a[nz])
    e = ex - 1
    frac = np.rint((a[nz] / np.ldexp(1.0, e) - 1.0) * 8).astype(np.int64)
    out[nz] = ((e + 7) << 3 | frac).astype(np.uint8)
    return out | sign


def e4m3_decode(bits):
    bits = np.asarray(bits, dtype=np.uint8)
    s = np.where(bits & 0x80, -1.0, 1.0)
    E = (bits >> 3) & 0xF
    M = (bits & 7).astype(np.float64)
    val = np.where(E == 0, M * 2.0 ** -9, np.ldexp(1.0 + M / 8.0, E.astype(np.int64) - 7))
    val = np.where((E == 15) & (M == 7), np.nan, val)
    return s * val


def bf16_decode(bits):
    bits = np.asarray(bits, dtype=np.uint16)
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def fp8_row_scales(X):
    """FP32 scale per row: fp32(amax / 448), 1 for an all-zero row."""
    amax = np.max(np.abs(X), axis=1)
    s = (amax / E4M3_MAX).astype(np.float32)
    return np.where(amax == 0, np.float32(1.0), s)


def quantize_rows(X, dtype):
    """Stored codes, row scales (FP32 or None) and the dequantised X^ (FP64)."""
    X = np.asarray(X, dtype=np.float64)
    if dtype == "bf16":
        codes = bf16_bits(X)
        return codes, None, bf16_decode(codes)
    if dtype == "fp8":
        s = fp8_row_scales(X)
        codes = e4m3_bits(X / s.astype(np.float64)[:, None])
        return codes, s, e4m3_decode(codes) * s.astype(np.float64)[:, None]
    raise ValueError(dtype)
