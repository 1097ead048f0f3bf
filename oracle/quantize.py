"""Low-precision storage of transition rows, written from the format definitions.

The paper fixes no precision (Sec. IV runs in the framework's default).  A
reduced-precision variant stores each transition row r in BF16 or in FP8
E4M3 together with one FP32 scale s_r, and the MDP that is then solved is

    P'(r, j) = s_r * decode(q_rj),      s_r = 1 / sum_j decode(q_rj),

so every stored row sums to 1 again (up to the FP32 rounding of s_r).  The
formats:

* BF16: the upper 16 bits of an IEEE binary32 (1 sign, 8 exponent, 7
  fraction bits); encoding rounds to nearest, ties to even.
* FP8 E4M3 (the OCP "E4M3FN" format): 1 sign, 4 exponent bits with bias 7,
  3 fraction bits; exponent field 0 is subnormal (value m * 2^-9); the code
  S.1111.111 is NaN; there are no infinities; the largest finite value is
  448.  Encoding rounds to nearest, ties to even, and saturates at 448.
  Before encoding, row r is multiplied by the power of two alpha_r =
  2^(7 - E_r), E_r the binary exponent of the row's largest magnitude, so the
  largest entry lands in [128, 256) and the scaling is exact (E_r is
  clamped to [-100, 127], which only rows of tiny entries reach); alpha_r
  cancels in s_r.

Test infrastructure only (see the package docstring).
"""

import numpy as np

BF16 = "bf16"
FP8 = "fp8"


# ------------------------------------------------------------ BF16

def bf16_encode(x):
    """float32 array -> uint16 codes, round to nearest even (NaN -> 0x7FC0)."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) & 0xFFFF
    r = np.where(nan, (u >> 16) | 0x40, r)
    return r.astype(np.uint16)


def bf16_decode(q):
    """uint16 codes -> float64 (exact)."""
    u = np.asarray(q, dtype=np.uint16).astype(np.uint32) << 16
    with np.errstate(invalid="ignore"):
        return u.view(np.float32).astype(np.float64)


# ------------------------------------------------------------ FP8 E4M3

def e4m3_decode(q):
    """uint8 codes -> float64 (exact), NaN for S.1111.111."""
    q = np.asarray(q, dtype=np.uint8).astype(np.int64)
    sign = np.where(q >> 7, -1.0, 1.0)
    e = (q >> 3) & 0xF
    m = q & 0x7
    normal = (1.0 + m / 8.0) * np.exp2(e - 7.0)
    sub = m * 2.0 ** -9
    v = np.where(e == 0, sub, normal)
    v = np.where((e == 15) & (m == 7), np.nan, v)
    return sign * v


def e4m3_encode(x):
    """float32 array -> uint8 codes: nearest value, ties to the even code,
    saturating at 448 (NaN -> 0x7F)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.int64)
    sign = (u >> 31) << 7
    a = u & 0x7FFFFFFF
    nan = a > 0x7F800000
    exp = (a >> 23) - 127
    frac = a & 0x7FFFFF
    # normal results: exponent >= -6; keep 3 fraction bits, round the other 20
    base = ((exp + 7) << 3) | (frac >> 20)
    rem = frac & 0xFFFFF
    up = (rem > 0x80000) | ((rem == 0x80000) & ((base & 1) == 1))
    normal_code = base + up
    # below 2^-6: multiples of 2^-9 (exact scaling, then round half to even)
    scaled = np.abs(x.astype(np.float64)) * 512.0
    with np.errstate(invalid="ignore"):
        sub_code = np.rint(np.where(exp >= -6, 0.0, scaled)).astype(np.int64)  # half to even
    code = np.where(exp >= -6, normal_code, sub_code)
    code = np.minimum(code, 0x7E)  # saturate at 448 (and +inf)
    code = np.where(nan, 0x7F, code)
    return (code | sign).astype(np.uint8)


# ------------------------------------------------------------ rows

def decode(q, dtype):
    return bf16_decode(q) if dtype == BF16 else e4m3_decode(q)


def _row_prescale(rows32):
    """alpha_r = 2^(7 - E_r) for FP8 (E_r the exponent of the largest
    magnitude of the row, from its binary32 bits); 1 for an all-zero row."""
    amax = np.max(np.abs(rows32), axis=1).astype(np.float32)
    e = ((amax.view(np.uint32) >> 23) & 0xFF).astype(np.int64) - 127
    e = np.clip(e, -100, 127)  # keeps alpha finite for (invalid) rows of tiny entries
    alpha = np.exp2((7 - e).astype(np.float64))
    return np.where(amax > 0, alpha, 1.0).astype(np.float32)


def quantize_rows(rows32, dtype):
    """rows32: float32 [rows, len].  Returns (codes [rows, len] uint16 or
    uint8, scale float32 [rows]) with scale_r = 1 / sum_j decode(q_rj) (0 for
    a row whose codes sum to 0)."""
    rows32 = np.ascontiguousarray(rows32, dtype=np.float32)
    if dtype == BF16:
        q = bf16_encode(rows32)
    elif dtype == FP8:
        alpha = _row_prescale(rows32)
        q = e4m3_encode((rows32 * alpha[:, None]).astype(np.float32))
    else:
        raise ValueError("dtype must be 'bf16' or 'fp8'")
    sums = decode(q, dtype).sum(axis=1)
    with np.errstate(divide="ignore"):
        scale = np.where(sums > 0, 1.0 / sums, 0.0).astype(np.float32)
    return q, scale


def dequantized(q, scale, dtype):
    """The stored rows as FP64: scale_r * decode(q_rj)."""
    return scale.astype(np.float64)[:, None] * decode(q, dtype)
