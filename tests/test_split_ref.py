"""Pins of the split reference (precision form) against exact arithmetic."""
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import core, split_ref
from paper_1306_4161_amd import inputs


@pytest.mark.parametrize("fmt", ["bf16", "e4m3", "int8"])
def test_digits_are_small_exact_integers(fmt):
    h, t = split_ref.FORMATS[fmt]
    X = inputs.exponent_spread(40, 64, 3, sigma=4.0)
    e = split_ref.exponents(X, axis=1)
    D = split_ref.digits(X, e, 7, fmt, axis=1)
    assert np.array_equal(D, np.rint(D))
    assert np.abs(D[0]).max() <= 2 ** h
    assert np.abs(D[1:]).max() <= 2 ** (t - 1)
    if fmt == "int8":
        # after the carry pass: the first digit in [-64, 65], the later in
        # [-128, 127], the int8 range
        assert np.abs(D[0]).max() <= 65
        assert D[1:].max() <= 127 and D[1:].min() >= -128
        back = D.astype(np.int8).astype(np.float64)
    else:
        dt = torch.bfloat16 if fmt == "bf16" else torch.float8_e4m3fn
        back = torch.from_numpy(D).to(dt).to(torch.float64).numpy()
    assert np.array_equal(back, D)


def test_int8_carries_worked_by_hand():
    # Rows [x, 1] have e = 0 (the 1), so x 2^6 is the first rounding.
    # x = 1/2 + 2^-7: x 2^6 = 32.5 -> 32 (half to even), remainder 1/2,
    # next 1/2 x 2^8 = 128 -> carried: digits 33, -128, 0.  With one digit
    # there is nothing to carry: 32.  The negative -32.5 -> -32 leaves -1/2,
    # next -128 fits: -32, -128, 0.
    # x = 2751999 / 2^24: x 2^6 = 10 + 130559/2^18 -> 10; the remainder
    # x 2^8 = 127 + 511/1024 -> 127; then 511/1024 x 2^8 = 127.75 -> 128:
    # the last digit carries into the 127, which carries into the 10:
    # digits 11, -128, -128 (two digits: 10, 127, no carry).
    x2 = 2751999 / 2.0 ** 24
    X = np.array([[0.5 + 2.0 ** -7, 1.0], [-(0.5 + 2.0 ** -7), 1.0], [x2, 1.0]])
    e = split_ref.exponents(X, axis=1)
    assert list(e) == [0, 0, 0]
    D3 = split_ref.digits(X, e, 3, "int8", axis=1)
    assert list(D3[:, 0, 0]) == [33, -128, 0]
    assert list(D3[:, 1, 0]) == [-32, -128, 0]
    assert list(D3[:, 2, 0]) == [11, -128, -128]
    assert list(D3[:, 0, 1]) == [64, 0, 0]
    assert list(split_ref.digits(X, e, 1, "int8", axis=1)[:, 0, 0]) == [32]
    assert list(split_ref.digits(X, e, 2, "int8", axis=1)[:, 2, 0]) == [10, 127]
    # the carries keep the value: x minus the digits is the last remainder
    # (0 for the ties, -1/4 unit of the third digit for x2)
    rec = split_ref.reconstruct(D3, e, "int8", axis=1)
    assert rec[0, 0] == X[0, 0] and rec[1, 0] == X[1, 0]
    assert X[2, 0] - rec[2, 0] == -0.25 * 2.0 ** (-6 - 16)


def test_exponent_is_smallest_power_bound():
    X = np.array([[0.75, -0.1], [256.0, 3.0], [0.0, 0.0], [-2.0 ** -30, 1e-300]])
    e = split_ref.exponents(X, axis=1)
    assert list(e) == [0, 8, 0, -30]
    for row, ei in zip(X, e):
        mx = np.abs(row).max()
        if mx:
            assert mx <= 2.0 ** ei and mx > 2.0 ** (ei - 1)


@pytest.mark.parametrize("fmt", ["bf16", "e4m3", "int8"])
def test_reconstruction_exact_and_remainder_bound(fmt):
    h, t = split_ref.FORMATS[fmt]
    X = inputs.uniform(16, 48, 11)
    e = split_ref.exponents(X, axis=1)
    # enough digits for every bit of every entry: exact reconstruction
    s_full = 2 + (53 + 60) // t
    D = split_ref.digits(X, e, s_full, fmt, axis=1)
    assert np.array_equal(split_ref.reconstruct(D, e, fmt, axis=1), X)
    # with s digits the remainder is at most 1/2 unit of the last digit
    for s in range(1, 7):
        Ds = split_ref.digits(X, e, s, fmt, axis=1)
        for i in range(X.shape[0]):
            for j in range(0, X.shape[1], 7):
                exact = Fraction(float(X[i, j]))
                approx = sum(Fraction(int(Ds[l, i, j])) * Fraction(2) ** (int(e[i]) - h - t * l)
                             for l in range(s))
                bound = Fraction(2) ** (int(e[i]) - h - t * (s - 1)) / 2
                assert abs(exact - approx) <= bound


def test_integers_up_to_256_are_one_bf16_digit():
    X = inputs.integer_valued(10, 30, 4, 8)
    X[0, 0] = 256.0
    e = split_ref.exponents(X, axis=1)
    D = split_ref.digits(X, e, 3, "bf16", axis=1)
    assert np.all(e <= 8)
    assert np.array_equal(np.ldexp(D[0], e[:, None] - 8), X)
    assert not D[1:].any()


def test_integers_up_to_64_are_one_int8_digit():
    X = inputs.integer_valued(10, 30, 4, 6)
    X[0, 0] = -64.0
    e = split_ref.exponents(X, axis=1)
    D = split_ref.digits(X, e, 3, "int8", axis=1)
    assert np.all(e <= 6)
    assert np.array_equal(np.ldexp(D[0], e[:, None] - 6), X)
    assert not D[1:].any()


def test_column_split_is_row_split_of_transpose():
    X = inputs.exponent_spread(24, 20, 9)
    ec = split_ref.exponents(X, axis=0)
    er = split_ref.exponents(X.T, axis=1)
    assert np.array_equal(ec, er)
    assert np.array_equal(split_ref.digits(X, ec, 5, "bf16", axis=0),
                          np.transpose(split_ref.digits(X.T, er, 5, "bf16", axis=1), (0, 2, 1)))


def test_pairs_triangular_count():
    for s in range(1, 9):
        p = split_ref.pairs(s)
        assert len(p) == s * (s + 1) // 2
        assert all(a + b <= s + 1 for a, b in p)


def test_truncated_product_exact_cases():
    # integer operands with |a| <= 256: one digit, nothing truncated -> exact
    A = inputs.integer_valued(6, 40, 1, 8)
    B = inputs.integer_valued(40, 5, 2, 8)
    rows, cols = np.meshgrid(np.arange(6), np.arange(5), indexing="ij")
    v = split_ref.truncated_entries(A, B, 16, 1, "bf16", rows.ravel(), cols.ravel())
    assert np.array_equal(v, core.exact_product(A, B).ravel())
    # entries bounded away from zero need <= 7 BF16 digits; with s = 13 every
    # nonzero digit pair is kept, so the truncated product is the exact one
    r = np.random.default_rng(3)
    A = r.uniform(2.0 ** -10, 1, (4, 24)) * r.choice([-1, 1], (4, 24))
    B = r.uniform(2.0 ** -10, 1, (24, 3)) * r.choice([-1, 1], (24, 3))
    rows, cols = np.meshgrid(np.arange(4), np.arange(3), indexing="ij")
    v = split_ref.truncated_entries(A, B, 8, 13, "bf16", rows.ravel(), cols.ravel())
    assert np.array_equal(v, core.exact_product(A, B).ravel())


def test_truncation_error_shrinks_with_slices():
    A = inputs.uniform(8, 64, 5)
    B = inputs.uniform(64, 8, 6)
    rows, cols = np.meshgrid(np.arange(8), np.arange(8), indexing="ij")
    rows, cols = rows.ravel(), cols.ravel()
    E = core.exact_product(A, B).ravel()
    S = (np.abs(A) @ np.abs(B)).ravel()
    prev = np.inf
    for s in range(2, 8):
        v = split_ref.truncated_entries(A, B, 32, s, "bf16", rows, cols)
        err = np.max(np.abs(v - E) / S)
        # per k-term the dropped part is at most about (s+2) 2^-(8+9(s-1)) of 2^(e+f)
        assert err <= (s + 2) * 2.0 ** (-8 - 9 * (s - 1)) * 64 / S.min() * 2 + 1e-16
        assert err <= prev or err < 1e-16
        prev = err
    assert prev < 1e-15


def test_int8_truncated_product_exact_and_error_shrinks():
    # integer operands with |a| <= 64: one INT8 digit, nothing truncated
    A = inputs.integer_valued(6, 40, 1, 6)
    B = inputs.integer_valued(40, 5, 2, 6)
    rows, cols = np.meshgrid(np.arange(6), np.arange(5), indexing="ij")
    v = split_ref.truncated_entries(A, B, 16, 1, "int8", rows.ravel(), cols.ravel())
    assert np.array_equal(v, core.exact_product(A, B).ravel())
    # general entries: error within the dropped part, shrinking by about 2^-8 per slice
    A = inputs.uniform(8, 64, 5)
    B = inputs.uniform(64, 8, 6)
    rows, cols = np.meshgrid(np.arange(8), np.arange(8), indexing="ij")
    rows, cols = rows.ravel(), cols.ravel()
    E = core.exact_product(A, B).ravel()
    S = (np.abs(A) @ np.abs(B)).ravel()
    prev = np.inf
    for s in range(2, 9):
        v = split_ref.truncated_entries(A, B, 32, s, "int8", rows, cols)
        err = np.max(np.abs(v - E) / S)
        assert err <= (s + 2) * 2.0 ** (-6 - 8 * (s - 1)) * 64 / S.min() * 2 + 1e-16
        assert err <= prev or err < 1e-16
        prev = err
    assert prev < 1e-15
