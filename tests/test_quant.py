"""Pins for the index's reduced-precision encodings (CPU only).

The library's host quantisers (used at index build) are compared with references written
here from the format definitions, not from the library:
* BF16: the top 16 bits of the FP32 pattern, rounded to nearest with ties to the even
  kept pattern (decided by the 16 discarded bits);
* FP8 e4m3fn: sign, 4 exponent bits with bias 7, 3 mantissa bits, subnormals m * 2^-9,
  no infinities, 0x7f / 0xff are NaN, largest finite 448; encoding rounds to the nearest
  representable value with ties to the even code and saturates at +-448.
"""
import math
import struct

import numpy as np
import pytest

import paper_2511_22460_amd as E


def f32_bits(x):
    return struct.unpack("<I", struct.pack("<f", x))[0]


def bits_f32(b):
    return struct.unpack("<f", struct.pack("<I", b & 0xffffffff))[0]


def ref_bf16(x):
    b = f32_bits(x)
    hi, lo = b >> 16, b & 0xffff
    if lo > 0x8000 or (lo == 0x8000 and (hi & 1)):
        hi += 1
    return hi & 0xffff


def ref_fp8_value(code):
    s, e, m = code >> 7, (code >> 3) & 15, code & 7
    if e == 15 and m == 7:
        return float("nan")
    v = m * 2.0 ** -9 if e == 0 else (1 + m / 8) * 2.0 ** (e - 7)
    return -v if s else v


FP8_TABLE = [(ref_fp8_value(c), c) for c in range(128) if not math.isnan(ref_fp8_value(c))]


def ref_fp8_encode(x):
    sign = 0x80 if math.copysign(1.0, x) < 0 else 0
    a = abs(x)
    best = None
    for v, c in FP8_TABLE:                     # non-negative values, codes 0x00..0x7e
        d = abs(v - a)
        if best is None or d < best[0] or (d == best[0] and (c & 1) == 0 and (best[1] & 1)):
            best = (d, c)
    if a > 448:
        return sign | 0x7e
    return sign | best[1]


def test_fp8_decode_all_codes():
    codes = np.arange(256, dtype=np.uint8)
    got = E.dequantize_fp8(codes)
    for c in range(256):
        want = ref_fp8_value(c)
        if math.isnan(want):
            assert math.isnan(got[c]), c
        else:
            assert got[c] == np.float32(want), (c, got[c], want)
    assert got[0x7e] == 448.0 and got[0x08] == 2.0 ** -6 and got[0x01] == 2.0 ** -9


def test_fp8_encode_roundtrip_and_halfway_cases():
    vals = sorted(v for v, _ in FP8_TABLE)
    xs = list(vals)
    # every halfway point between neighbours (ties to even code), and points just off it
    for lo, hi in zip(vals, vals[1:]):
        mid = (lo + hi) / 2
        xs += [mid, np.nextafter(np.float32(mid), np.float32(0)), np.nextafter(np.float32(mid), np.float32(1e9))]
    xs += [448.0, 449.0, 463.9, 464.0, 1e6, 2.0 ** -10, 2.0 ** -11, 3 * 2.0 ** -11]
    rng = np.random.default_rng(0)
    xs += list(rng.normal(0, 30, 2000)) + list(rng.normal(0, 0.01, 500))
    xs = np.array(xs + [-x for x in xs], dtype=np.float32)
    got = E.quantize_fp8(xs)
    for x, c in zip(xs, got):
        assert c == ref_fp8_encode(float(x)), (float(x), int(c), ref_fp8_encode(float(x)))


def test_fp8_scale_applied_before_rounding():
    x = np.array([0.5, -0.25, 3.0], np.float32)
    c = E.quantize_fp8(x, scale=3.0 / 448)
    assert E.dequantize_fp8(c)[2] == 448.0
    with pytest.raises(E.EbrError):
        E.quantize_fp8(x, scale=0.0)


def test_bf16_round_to_nearest_even():
    rng = np.random.default_rng(1)
    xs = list(rng.normal(0, 1, 3000).astype(np.float32))
    # exact ties: low 16 bits 0x8000 with odd and even kept parts; just above/below ties
    for hi in (0x3f80, 0x3f81, 0xbf80, 0xbf81, 0x0001, 0x7f7e):
        for lo in (0x8000, 0x7fff, 0x8001, 0x0000, 0xffff):
            xs.append(bits_f32((hi << 16) | lo))
    xs = np.array(xs, dtype=np.float32)
    got = E.quantize_bf16(xs)
    for x, h in zip(xs, got):
        assert h == ref_bf16(float(x)), (float(x), hex(int(h)), hex(ref_bf16(float(x))))
    with pytest.raises(E.EbrError):
        E.quantize_bf16(np.array([np.inf], np.float32))
