"""Pins for the two-term split of Sec. III.A (Eqs. dualRep, splitStyle)."""
import struct

import numpy as np
import pytest

from oracle import zf_oracle as O


def _f32(x):
    return struct.unpack("<f", struct.pack("<f", x))[0]


def _bits(x):
    return struct.unpack("<I", struct.pack("<f", x))[0]


def _from_bits(u):
    return struct.unpack("<f", struct.pack("<I", u & 0xFFFFFFFF))[0]


def _nearest_bf16_bruteforce(x):
    """Nearest BF16 to the FP32 number x, ties to the even pattern, found by
    comparing the two BF16 neighbours bracketing x (pure Python)."""
    if x != x:
        return None
    u = _bits(x)
    lo_pat = u >> 16                      # truncation toward zero
    hi_pat = lo_pat + 1                   # next BF16 away from zero
    a = _from_bits(lo_pat << 16)
    b = _from_bits(hi_pat << 16) if (hi_pat & 0x7FFF) <= 0x7F80 else float("inf") * (1 if a >= 0 else -1)
    da, db = abs(x - a), abs(b - x)
    if da < db:
        return a
    if db < da:
        return b
    return a if lo_pat % 2 == 0 else b


def _edge_values():
    v = [0.0, -0.0, 1.0, -1.0, 2.0 ** -126, -(2.0 ** -126), 2.0 ** -149, 3.0 * 2.0 ** -140,
         3.3895313892515355e38, 1.0e-30, 65504.0, 6.1e-5, 5.96e-8]
    for base in (1.0, 1.5, 0.75, 1e-3, 1e3, 3.0e-20):
        b = _bits(_f32(base))
        hi16 = b & 0xFFFF0000
        for low in (0x7FFF, 0x8000, 0x8001, 0x0001, 0xFFFF):
            v.append(_from_bits(hi16 | low))
            v.append(-_from_bits(hi16 | low))
        # tie with odd bf16 mantissa
        v.append(_from_bits((hi16 + 0x10000) | 0x8000))
    return np.array(v, dtype=np.float32)


def test_bf16_rounding_edge_values():
    xs = _edge_values()
    hi, lo = O.split(xs.astype(np.float64), "bf16")
    for x, h in zip(xs.tolist(), hi.tolist()):
        assert h == _nearest_bf16_bruteforce(x), x
    # the bit view works for every produced value
    O.bf16_bits(hi)
    O.bf16_bits(lo)


def test_bf16_rounding_random_vs_bruteforce():
    rng = np.random.default_rng(0)
    xs = (rng.standard_normal(4000) * np.exp(rng.uniform(-30, 30, 4000))).astype(np.float32)
    hi, _ = O.split(xs.astype(np.float64), "bf16")
    for x, h in zip(xs.tolist(), hi.tolist()):
        assert h == _nearest_bf16_bruteforce(x)


@pytest.mark.parametrize("fmt,u", [("bf16", 2.0 ** -8), ("fp16", 2.0 ** -11)])
def test_split_error_bound(fmt, u):
    """|A - A^(h) - A^(l)| <= u^2 |A| with A = FP32[A] (Sec. III.A), in the normal range."""
    rng = np.random.default_rng(1)
    a = rng.uniform(-1, 1, 20000) * (8.0 if fmt == "fp16" else 1e10) \
        * (1 if fmt == "fp16" else np.exp(rng.uniform(-40, 0, 20000)))
    if fmt == "fp16":
        a = a[np.abs(a) > 2.0 ** -2]            # keep the low part above FP16's normal range
    a32 = O.to_fp32(a).astype(np.float64)
    hi, lo = O.split(a, fmt)
    err = np.abs(a32 - hi.astype(np.float64) - lo.astype(np.float64))
    assert np.all(err <= u * u * np.abs(a32))
    # the residual A - FP32[A^(h)] is exact in FP32
    r = a32 - hi.astype(np.float64)
    assert np.all(r.astype(np.float32).astype(np.float64) == r)


def test_fp64_to_fp32_is_rne():
    # 1 + 2^-24 is a tie between 1 and 1 + 2^-23: RNE keeps 1; 1 + 3*2^-24 goes up
    a = np.array([1 + 2.0 ** -24, 1 + 3 * 2.0 ** -24, -(1 + 2.0 ** -24)])
    np.testing.assert_array_equal(O.to_fp32(a), np.array([1.0, 1 + 2.0 ** -22, -1.0], np.float32))


def test_split_product_drops_only_low_low():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((16, 16))
    B = rng.standard_normal((16, 16))
    ah, al = O.split(A)
    bh, bl = O.split(B)
    full = (ah.astype(float) + al) @ (bh.astype(float) + bl)
    np.testing.assert_allclose(O.split_product(ah, al, bh, bl) + al.astype(float) @ bl, full,
                               rtol=1e-13, atol=1e-13)
