"""Pins of the oracle's BF16 / FP8 E4M3 row quantiser (CPU).

References other than the oracle itself: torch's own bfloat16 and
float8_e4m3fn conversions (library routines), brute force over every code,
and properties fixed by the format definitions.
"""
import numpy as np
import pytest
import torch

from oracle import quantize as qz


def _rng(seed):
    return np.random.Generator(np.random.Philox(seed))


def _spread(n, seed, lo=-14, hi=9):
    """Random float32 magnitudes spread over binary exponents [lo, hi)."""
    g = _rng(seed)
    return (g.random(n) * np.exp2(g.integers(lo, hi, n))).astype(np.float32)


# ------------------------------------------------------------ BF16

def test_bf16_encode_matches_torch():
    x = np.concatenate([_spread(20000, 1, -140, 120), -_spread(2000, 2, -30, 30),
                        np.array([0.0, -0.0, 1.0, 3.0e38, 1e-45, np.inf, -np.inf],
                                 dtype=np.float32)]).astype(np.float32)
    # exact ties: low 16 bits 0x8000, with even and odd kept parts
    u = _rng(3).integers(0x00800000, 0x7F000000, 4000, dtype=np.uint32)
    ties = ((u & 0xFFFF0000) | 0x8000).astype(np.uint32).view(np.float32)
    x = np.concatenate([x, ties])
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(qz.bf16_encode(x), ref)


def test_bf16_decode_is_exact_and_inverts_encode():
    codes = np.arange(0, 1 << 16, dtype=np.uint32).astype(np.uint16)
    finite = (codes & 0x7F80) != 0x7F80
    dec = qz.bf16_decode(codes)
    ref = torch.from_numpy(codes.view(np.int16)).view(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(dec[finite], ref[finite])
    again = qz.bf16_encode(dec[finite].astype(np.float32))
    assert np.array_equal(again, codes[finite])


# ------------------------------------------------------------ FP8 E4M3

def test_e4m3_decode_table_matches_torch_and_definition():
    codes = np.arange(256, dtype=np.uint8)
    dec = qz.e4m3_decode(codes)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(np.isnan(dec), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.array_equal(dec[ok], ref[ok])
    # fixed points of the definition
    assert dec[0x7E] == 448.0 and dec[0x08] == 2.0 ** -6 and dec[0x01] == 2.0 ** -9
    assert dec[0x00] == 0.0 and np.isnan(dec[0x7F]) and np.isnan(dec[0xFF])
    assert dec[0x38] == 1.0 and dec[0xB8] == -1.0
    assert np.all(np.diff(dec[:0x7F]) > 0)  # monotone over the finite positive codes


def _nearest_code(x):
    """Brute force: the finite positive code nearest to |x| (ties to the even
    code), saturating at 448."""
    vals = qz.e4m3_decode(np.arange(0x7F, dtype=np.uint8))
    out = np.empty(len(x), dtype=np.uint8)
    for i, v in enumerate(np.abs(x.astype(np.float64))):
        d = np.abs(vals - v)
        best = np.flatnonzero(d == d.min())
        c = best[0] if len(best) == 1 else [b for b in best if b % 2 == 0][0]
        out[i] = c | (0x80 if np.signbit(x[i]) else 0)
    return out


def test_e4m3_encode_is_nearest_with_ties_to_even():
    x = np.concatenate([_spread(3000, 4, -12, 9), -_spread(300, 5, -12, 9)])
    # exact midpoints between neighbouring codes
    vals = qz.e4m3_decode(np.arange(0x7F, dtype=np.uint8))
    mids = ((vals[:-1] + vals[1:]) / 2).astype(np.float32)
    x = np.concatenate([x, mids, vals.astype(np.float32)]).astype(np.float32)
    assert np.array_equal(qz.e4m3_encode(x), _nearest_code(x))


def test_e4m3_encode_matches_torch_in_range():
    x = np.concatenate([_spread(50000, 6, -14, 9), -_spread(5000, 7, -14, 9)])
    x = x[np.abs(x) < 464].astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(qz.e4m3_encode(x), ref)


def test_e4m3_saturates_and_keeps_nan():
    x = np.array([448.0, 449.0, 464.0, 1e6, np.inf, -1e6, np.nan], dtype=np.float32)
    assert qz.e4m3_encode(x).tolist() == [0x7E, 0x7E, 0x7E, 0x7E, 0x7E, 0xFE, 0x7F]


# ------------------------------------------------------------ rows

@pytest.mark.parametrize("dtype", [qz.BF16, qz.FP8])
def test_quantized_rows_sum_to_one(dtype):
    g = _rng(8)
    rows = g.gamma(0.1, size=(64, 1000))
    rows = (rows / rows.sum(axis=1, keepdims=True)).astype(np.float32)
    q, s = qz.quantize_rows(rows, dtype)
    Pq = qz.dequantized(q, s, dtype)
    assert np.all(np.abs(Pq.sum(axis=1) - 1.0) <= 2.0 ** -23)
    # the stored MDP stays close to the original: per-entry relative error of
    # the format (2^-8 BF16, 2^-4 FP8) plus the renormalisation, or the
    # absolute floor where entries underflow
    tol = (2.0 ** -7 if dtype == qz.BF16 else 2.0 ** -3) * rows + 2.0 ** -16
    assert np.all(np.abs(Pq - rows) <= tol + 1e-3 * rows.max(axis=1, keepdims=True) *
                  (dtype == qz.FP8))


def test_fp8_prescale_puts_the_row_maximum_in_128_256():
    # before rounding the scaled maximum lies in [128, 256); rounding may carry it to 256
    g = _rng(9)
    rows = (g.random((50, 33)) * np.exp2(g.integers(-20, 5, (50, 1)))).astype(np.float32)
    q, _ = qz.quantize_rows(rows, qz.FP8)
    top = qz.e4m3_decode(q).max(axis=1)
    assert np.all((top >= 128.0) & (top <= 256.0))
    scaled = rows.max(axis=1) * qz._row_prescale(rows)
    assert np.all((scaled >= 128.0) & (scaled < 256.0))
    q0, s0 = qz.quantize_rows(np.zeros((2, 8), dtype=np.float32), qz.FP8)
    assert np.all(q0 == 0) and np.all(s0 == 0.0)
