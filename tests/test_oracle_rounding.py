"""Pins of the oracle's BF16 / FP8 E4M3FN rounding.

Brute force: the nearest representable value is found by searching the full
table of codes (decoded by torch), ties going to the even code. The torch
casts from float32 are a second, library reference.
"""
import numpy as np
import pytest
import torch

import oracle as O


def _table(dtype, nbits):
    codes = torch.arange(2**nbits, dtype=torch.int32)
    if nbits == 16:
        vals = codes.to(torch.int16).view(torch.bfloat16).to(torch.float64).numpy()
    else:
        vals = codes.to(torch.uint8).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    codes = codes.numpy()
    ok = np.isfinite(vals)
    return vals[ok], codes[ok]


def _nearest(x, vals, codes):
    d = np.abs(vals - x)
    best = d.min()
    cand = np.where(d == best)[0]
    if len(cand) > 1:
        # ties: the code with an even mantissa (last bit 0); drop -0 duplicates
        cand = [c for c in cand if codes[c] % 2 == 0] or list(cand)
    v = vals[cand[0]]
    return v


@pytest.fixture(scope="module")
def bf16_table():
    return _table(torch.bfloat16, 16)


@pytest.fixture(scope="module")
def fp8_table():
    return _table(torch.float8_e4m3fn, 8)


def _samples(rng, lo_exp, hi_exp, n):
    mant = rng.uniform(1.0, 2.0, n)
    ex = rng.integers(lo_exp, hi_exp, n)
    sign = rng.choice([-1.0, 1.0], n)
    return sign * np.ldexp(mant, ex)


def test_bf16_bruteforce(bf16_table):
    vals, codes = bf16_table
    rng = np.random.default_rng(0)
    xs = list(_samples(rng, -133, 127, 1500))
    # exact midpoints between neighbours, and a hair either side of them
    mids = (vals[1:200:3] + vals[2:201:3]) / 2
    xs += list(mids) + list(np.nextafter(mids, np.inf)) + list(np.nextafter(mids, -np.inf))
    for x in xs:
        assert O.round_bf16(x) == _nearest(x, vals, codes), x


def test_bf16_matches_torch_cast_from_f32():
    rng = np.random.default_rng(1)
    x = np.concatenate([_samples(rng, -140, 127, 5000),
                        np.float32(rng.normal(size=2000))]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = O.round_bf16(x.astype(np.float64))
    assert np.array_equal(got, want)


def test_bf16_overflow_to_inf():
    big = float(np.float32(3.4e38))   # above (2 - 2^-8) * 2^127
    assert O.round_bf16(big) == np.inf and O.round_bf16(-big) == -np.inf


def test_fp8_bruteforce(fp8_table):
    vals, codes = fp8_table
    rng = np.random.default_rng(2)
    xs = list(_samples(rng, -12, 9, 3000))
    svals = np.unique(vals)
    mids = (svals[:-1] + svals[1:]) / 2
    xs += list(mids) + list(np.nextafter(mids, np.inf)) + list(np.nextafter(mids, -np.inf))
    for x in xs:
        want = float(np.clip(_nearest(x, vals, codes), -448, 448)) if abs(x) <= 448 else \
            float(np.sign(x) * 448)
        assert O.round_fp8(x) == want, x


def test_fp8_matches_torch_cast_in_range():
    rng = np.random.default_rng(3)
    x = np.float32(rng.uniform(-448, 448, 20000) * rng.choice([1, 1e-2, 1e-4], 20000))
    want = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(O.round_fp8(x.astype(np.float64)), want)


def test_fp8_saturates():
    assert O.round_fp8(1e6) == 448.0 and O.round_fp8(-470.0) == -448.0
    assert O.round_fp8(460.0) == 448.0
