"""Reference LU factorisation without pivoting -- TEST INFRASTRUCTURE ONLY.

The paper names LU (and QR) factorisation as a workload for the
hierarchical panel updates (Sec. VI): a blocked LU spends its time in the
trailing-matrix update A22 <- A22 - L21 U12, which is the local update
C += A_panel x B_panel of Sec. II-A with C = A22.  What the factorisation
computes has a plain definition, written out here as textbook Gaussian
elimination (no pivoting, for matrices where every leading principal minor
is nonzero, e.g. diagonally dominant ones):

    for k = 0 .. n-1:
        l_ik = a_ik / a_kk                       (i > k)
        a_ij = a_ij - l_ik a_kj                  (i > k, j > k)

so that A = L U with L unit lower triangular (the l_ik) and U upper
triangular (the final a_kj, j >= k).  The result is returned packed: the
strict lower part holds L, the upper part (with the diagonal) holds U.  One
rounding per operation, in the order above (no fused multiply-add).

Functions
  lu_nopivot(A)          packed LU by the elimination above (O(n^3) in
                         numpy row operations: n up to about 1000).
  unpack(LU)             (L, U) as dense matrices.
  residual_sampled(LU, A, rows, cols)
                         |(L U)_ij - a_ij| and (|L||U|)_ij at the sampled
                         entries, with (L U)_ij by Dot2 (core.sampled), for
                         the backward-error check |L U - A| <= gamma_n |L||U|
                         of any n-step elimination (Higham, Accuracy and
                         Stability, Thm. 9.3).

Pinned by tests/test_lu_ref.py: a 3 x 3 example worked by hand
(tests/golden/lu_3x3.txt), exact recovery of integer factors with power-of-
two pivots, agreement with LAPACK's partial-pivoting LU on matrices whose
columns are strictly diagonally dominant (where partial pivoting makes no
swap), det A = prod u_kk, and the backward-error bound.
"""
from __future__ import annotations

import numpy as np

from . import core


def lu_nopivot(A) -> np.ndarray:
    A = np.array(A, dtype=np.float64, copy=True)
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("square matrix expected")
    for k in range(n):
        piv = A[k, k]
        if piv == 0.0:
            raise ZeroDivisionError("zero pivot at step %d: LU without pivoting does not exist" % k)
        A[k + 1:, k] = A[k + 1:, k] / piv
        # one rounding for the product, one for the difference
        A[k + 1:, k + 1:] = A[k + 1:, k + 1:] - np.multiply.outer(A[k + 1:, k], A[k, k + 1:])
    return A


def unpack(LU):
    LU = np.asarray(LU, dtype=np.float64)
    n = LU.shape[0]
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    return L, U


def residual_sampled(LU, A, rows, cols):
    L, U = unpack(LU)
    c, s = core.sampled(L, U, rows, cols)
    return np.abs(c - np.asarray(A)[rows, cols]), s
