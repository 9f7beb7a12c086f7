"""Pins of the LU oracle (oracle/lu_ref.py) against things other than itself."""
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import core, lu_ref
from paper_1306_4161_amd import inputs


def _golden(golden_dir):
    rows = {"A": [], "L": [], "U": []}
    with open(os.path.join(golden_dir, "lu_3x3.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            tag, *vals = line.split()
            rows[tag].append([float(v) for v in vals])
    return {k: np.array(v) for k, v in rows.items()}


def test_hand_worked_3x3(golden_dir):
    g = _golden(golden_dir)
    LU = lu_ref.lu_nopivot(g["A"])
    L, U = lu_ref.unpack(LU)
    assert np.array_equal(L, g["L"]) and np.array_equal(U, g["U"])
    assert np.array_equal(g["L"] @ g["U"], g["A"])


def _integer_factors(n, seed):
    # L0 unit lower with entries in {-1, 0, 1}, U0 upper with power-of-two
    # diagonal and small integers above: A = L0 U0 is exact in binary64, and
    # elimination recovers L0 and U0 exactly (every quotient by a power of two
    # and every partial Schur complement is a small dyadic number)
    rng = np.random.default_rng(seed)
    L0 = np.tril(rng.integers(-1, 2, size=(n, n)).astype(np.float64), -1) + np.eye(n)
    U0 = np.triu(rng.integers(-2, 3, size=(n, n)).astype(np.float64), 1)
    U0 += np.diag(rng.choice([-2.0, -1.0, 1.0, 2.0, 4.0], size=n))
    return L0, U0


@pytest.mark.parametrize("n", [1, 2, 7, 64, 129])
def test_integer_factors_recovered_exactly(n):
    L0, U0 = _integer_factors(n, 100 + n)
    A = L0 @ U0
    assert np.abs(A).max() < 2.0 ** 40
    L, U = lu_ref.unpack(lu_ref.lu_nopivot(A))
    assert np.array_equal(L, L0) and np.array_equal(U, U0)


@pytest.mark.parametrize("n", [5, 50, 300])
def test_agrees_with_partial_pivoting_when_no_row_swaps(n):
    # columns strictly diagonally dominant: partial pivoting keeps the
    # diagonal pivot at every step (the property is preserved by
    # elimination), so LAPACK's getrf returns P = I and the same factors
    A = inputs.uniform(n, n, 7 + n)
    A += np.diag(np.abs(A).sum(axis=0) + 1.0)
    P, Ls, Us = scipy.linalg.lu(A)
    assert np.array_equal(P, np.eye(n))
    L, U = lu_ref.unpack(lu_ref.lu_nopivot(A))
    scale = np.abs(L) @ np.abs(U)
    tol = 4 * core.gamma(n) * scale
    assert np.all(np.abs(L @ U - Ls @ Us) <= tol + 1e-300)
    assert np.allclose(L, Ls, rtol=0, atol=1e-12) and np.allclose(U, Us, rtol=1e-12, atol=1e-12)


def test_determinant_is_product_of_pivots():
    n = 40
    A = inputs.uniform(n, n, 3) + n * np.eye(n)
    U = np.triu(lu_ref.lu_nopivot(A))
    d_ref = np.linalg.det(A)
    assert abs(np.prod(np.diag(U)) - d_ref) <= 1e-12 * abs(d_ref)


@pytest.mark.parametrize("n", [16, 200])
def test_backward_error_bound(n):
    A = inputs.exponent_spread(n, n, 11, 1.0) + 4 * n * np.eye(n)
    LU = lu_ref.lu_nopivot(A)
    rows, cols = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    rows, cols = rows.ravel(), cols.ravel()
    r, s = lu_ref.residual_sampled(LU, A, rows, cols)
    assert np.all(r <= core.gamma(n) * s + 2 * core.U * np.abs(A[rows, cols]))


def test_zero_pivot_is_reported():
    with pytest.raises(ZeroDivisionError):
        lu_ref.lu_nopivot(np.array([[0.0, 1.0], [1.0, 0.0]]))
