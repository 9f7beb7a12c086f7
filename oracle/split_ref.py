"""Reference of the precision form's operand split (not part of the paper).

TEST INFRASTRUCTURE ONLY.  The precision form replaces the FP64 local update
by products of small-integer "digit" matrices in the spirit of the error-free
splitting of Ozaki, Ogita, Oishi and Rump ("Error-free transformations of
matrix multiplication by using fast routines of matrix multiplication and its
applications", Numer. Algorithms 59, 2012).  The rule written here is this
project's reading of that method for BF16 / FP8-e4m3 / INT8 digit planes:

  * Per outer panel (the M-wide k-range of one outer step), each row i of the
    A panel gets the exponent e_i = smallest integer with max_l |a_il| <= 2^e_i
    (0 for an all-zero row); each column j of the B panel likewise gets f_j.
  * x = a * 2^-e lies in [-1, 1].  The first digit is d_1 = rint(x * 2^h)
    and later digits d_l = rint(r_{l-1} * 2^t) of the running remainder
    r_l = r_{l-1} * 2^t - d_l (r_0 = x, first shift h), with rint = round half
    to even.  BF16 uses h = 8, t = 9; FP8-e4m3 uses h = 4, t = 5, so every
    digit is an integer with |d| <= 2^h (256 or 16), exactly representable in
    the narrow format.  INT8 uses h = 6, t = 8: the rounded digits lie in
    [-64, 64] (first) and [-128, 128] (later), and a carry pass over the s
    digits, from the last to the second, replaces a digit of 128 (or 129
    after a carry) by itself minus 256 and adds one to the digit before it.
    That keeps the value (256 units of digit l are one unit of digit l - 1)
    and the remainder, and leaves every later digit in [-128, 127] and the
    first in [-64, 65]: the range of int8.  The carries depend on s, so the
    first planes of an s-digit split can differ from a shorter split's.
    Every step is exact in binary64.
  * a = 2^e * (sum_{l<=s} d_l 2^-(h + t(l-1)) + r_s 2^-(h + t(s-1))) exactly,
    with |r_s| <= 1/2.
  * The product keeps the digit pairs (l1, l2) with l1 + l2 <= s + 1; pair
    (l1, l2) is scaled by 2^(e_i + f_j - 2h - t(l1 + l2 - 2)).

Functions
  exponents(X, axis)      per-row (axis=1) or per-column (axis=0) e.
  digits(X, e, s, fmt, axis)   the s digit planes (float64 holding integers).
  reconstruct(D, e, fmt, axis) sum of the planes back in binary64 (exact if
                          enough digits are kept).
  truncated_entries(A, B, M, s, fmt, rows, cols)
                          the exact value (Python integers, then one rounding)
                          of what the split product computes for the sampled
                          entries, summed over all outer panels.

Pinned by tests/test_split_ref.py: exact reconstruction with enough digits,
the remainder bound, digit range and integrality, exactness of the digits in
torch bfloat16 / float8_e4m3fn / int8, INT8 carries worked by hand (a tie, a
negative tie, a two-step cascade, and the count dependence), integer-valued
inputs as single digits, and brute-force exact products.  The choice of rule itself is a reading (the
paper has no precision form); parity of the split GPU path against this
reference is to the truncation bound plus FP64 accumulation error.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

FORMATS = {"bf16": (8, 9), "e4m3": (4, 5), "int8": (6, 8)}
CARRY = {"int8"}                        # formats whose digits take the carry pass


def exponents(X, axis: int) -> np.ndarray:
    """Smallest integer e with max |x| <= 2^e along `axis` (0 if all zero)."""
    X = np.asarray(X, dtype=np.float64)
    mx = np.max(np.abs(X), axis=axis) if X.size else np.zeros(X.shape[1 - axis])
    m, e = np.frexp(mx)                 # mx = m 2^e, m in [0.5, 1)
    e = e.astype(np.int64)
    e = np.where(m == 0.5, e - 1, e)    # exact powers of two: 2^(e-1) itself
    e = np.where(mx == 0, 0, e)
    return e


def digits(X, e, s: int, fmt: str, axis: int) -> np.ndarray:
    """Digit planes, shape (s,) + X.shape; axis=1: e per row, axis=0: per column."""
    h, t = FORMATS[fmt]
    X = np.asarray(X, dtype=np.float64)
    e = np.asarray(e, dtype=np.int64)
    ee = e[:, None] if axis == 1 else e[None, :]
    r = np.ldexp(X, -ee)                # exact: scaling by a power of two
    out = np.empty((s,) + X.shape, dtype=np.float64)
    shift = h
    for l in range(s):
        y = np.ldexp(r, shift)
        d = np.rint(y)
        out[l] = d
        r = y - d                       # exact: the fraction bits of y
        shift = t
    if fmt in CARRY:
        for l in range(s - 1, 0, -1):
            over = out[l] >= 128
            out[l] = np.where(over, out[l] - 256, out[l])
            out[l - 1] = out[l - 1] + over
    return out


def reconstruct(D, e, fmt: str, axis: int) -> np.ndarray:
    h, t = FORMATS[fmt]
    e = np.asarray(e, dtype=np.int64)
    ee = e[:, None] if axis == 1 else e[None, :]
    acc = np.zeros(D.shape[1:], dtype=np.float64)
    for l in range(D.shape[0] - 1, -1, -1):   # smallest first
        acc = acc + np.ldexp(D[l], -(h + t * l))
    return np.ldexp(acc, ee)


def pairs(s: int) -> list[tuple[int, int]]:
    """Kept digit pairs (1-based): l1 + l2 <= s + 1."""
    return [(l1, l2) for l1 in range(1, s + 1) for l2 in range(1, s + 1) if l1 + l2 <= s + 1]


def truncated_entries(A, B, M: int, s: int, fmt: str, rows, cols) -> np.ndarray:
    """Exact value of the truncated split product at (rows[t], cols[t]), rounded once."""
    h, t = FORMATS[fmt]
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    k = A.shape[1]
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    ur, ri = np.unique(rows, return_inverse=True)
    uc, ci = np.unique(cols, return_inverse=True)
    total = [Fraction(0)] * rows.size
    for g0 in range(0, k, M):
        g1 = min(g0 + M, k)
        ea = exponents(A[:, g0:g1], axis=1)[ur]
        fb = exponents(B[g0:g1, :], axis=0)[uc]
        DA = digits(A[ur, g0:g1], ea, s, fmt, axis=1).astype(np.int64)   # (s, |ur|, w)
        DB = digits(B[g0:g1][:, uc], fb, s, fmt, axis=0).astype(np.int64)  # (s, w, |uc|)
        for idx in range(rows.size):
            a = DA[:, ri[idx], :]          # (s, w)
            b = DB[:, :, ci[idx]]          # (s, w)
            P = a @ b.T                    # exact int64: |sum| <= w 2^(2h) << 2^63
            acc = 0
            for (l1, l2) in pairs(s):
                # common denominator 2^(2h + t(2s-2)); pair weight 2^-(2h + t(l1+l2-2))
                acc += int(P[l1 - 1, l2 - 1]) << (t * (2 * s - l1 - l2))
            scale = int(ea[ri[idx]] + fb[ci[idx]]) - 2 * h - t * (2 * s - 2)
            total[idx] += Fraction(acc) * (Fraction(2) ** scale)
    return np.array([float(v) for v in total], dtype=np.float64)
