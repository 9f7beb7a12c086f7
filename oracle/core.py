"""Plain FP64 oracle: binding of oracle.c plus exact brute force.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Functions
  gemm(A, B, C=None)      the plain definition c_ij = sum_k a_ik b_kj that SUMMA
                          and HSUMMA reach after n/b steps (Sec. II-A, Sec. III),
                          summed in increasing k with one rounding per operation.
                          With C given, accumulates (one local update step,
                          c_ij = c_ij + a_ik x b_kj, Sec. II-A).
  sampled(A, B, rows, cols)
                          entries of A*B by Dot2 (Ogita-Rump-Oishi 2005), as
                          accurate as a twice-working-precision dot product,
                          plus s_ij = sum_k |a_ik||b_kj|.
  freivalds(A, B, C_hat, x)
                          residual |C_hat x - A(Bx)| and the bound it must meet.
  exact_product(A, B)     exact rational A*B (fractions.Fraction), rounded to
                          nearest-even binary64: the reference that pins gemm
                          and sampled on tiny inputs.
  python_gemm(A, B)       the same sum as gemm, in pure Python floats, for
                          tiny inputs (pins the loop order of oracle.c).

Pinned by tests/test_oracle.py: exact brute force, pure-Python sums, identity,
diagonal, rank-1 and integer-valued operands, cancellation cases for Dot2.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# HSUMMA_ORACLE_SANITIZE=1: the AddressSanitizer / UndefinedBehaviorSanitizer
# build (liboracle_asan.so; the process must preload gcc's libasan)
_SANITIZE = os.environ.get("HSUMMA_ORACLE_SANITIZE") == "1"
_LIB_PATH = os.environ.get("HSUMMA_ORACLE_LIBRARY") or os.path.join(
    _HERE, "liboracle_asan.so" if _SANITIZE else "liboracle.so")
_lib = None

U = 2.0 ** -53  # unit roundoff of binary64


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (no BLAS, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    ):
        os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = [
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
            "-shared", "-fPIC", "-o", tmp, _SRC, "-lm",
        ]
        if _SANITIZE:
            cmd[1:1] = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        "-fno-omit-frame-pointer"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        i64, dp = ctypes.c_int64, ctypes.c_void_p
        lib.oracle_gemm.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, i64, ctypes.c_int]
        lib.oracle_gemm.restype = None
        lib.oracle_sampled.argtypes = [i64, dp, i64, dp, i64, i64, dp, dp, dp, dp]
        lib.oracle_sampled.restype = None
        lib.oracle_matvec2.argtypes = [i64, i64, dp, i64, dp, dp, dp]
        lib.oracle_matvec2.restype = None
        lib.oracle_dot2.argtypes = [i64, dp, i64, dp, i64, dp]
        lib.oracle_dot2.restype = ctypes.c_double
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    a = np.asarray(a)
    if a.dtype != np.float64 or not a.flags.c_contiguous:
        a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def threads() -> int:
    return int(_load().oracle_threads())


def gemm(A, B, C=None) -> np.ndarray:
    """C = A*B (C None) or C += A*B in place (C given); plain k-ordered sums."""
    lib = _load()
    A, B = _f64(A), _f64(B)
    m, k = A.shape
    k2, n = B.shape
    if k != k2:
        raise ValueError("inner dimensions differ")
    acc = 1
    if C is None:
        C = np.empty((m, n), dtype=np.float64)
        acc = 0
    elif C.dtype != np.float64 or C.shape != (m, n) or C.strides[1] != 8:
        raise ValueError("C must be float64 (m, n) with unit column stride")
    lib.oracle_gemm(m, n, k, _ptr(A), A.strides[0] // 8, _ptr(B), B.strides[0] // 8,
                    _ptr(C), C.strides[0] // 8, acc)
    return C


def gemm_view(A, B, C) -> None:
    """C += A*B where A, B, C may be row-strided views (unit column stride)."""
    lib = _load()
    for X in (A, B, C):
        if X.dtype != np.float64 or X.strides[1] != 8:
            raise ValueError("operands must be float64 with unit column stride")
    m, k = A.shape
    n = B.shape[1]
    lib.oracle_gemm(m, n, k, _ptr(A), A.strides[0] // 8, _ptr(B), B.strides[0] // 8,
                    _ptr(C), C.strides[0] // 8, 1)


def dot2(x, y) -> tuple[float, float]:
    """(Dot2(x, y), sum |x_i y_i|)."""
    lib = _load()
    x, y = _f64(x), _f64(y)
    s = ctypes.c_double()
    r = lib.oracle_dot2(x.size, _ptr(x), 1, _ptr(y), 1, ctypes.byref(s))
    return r, s.value


def sampled(A, B, rows, cols) -> tuple[np.ndarray, np.ndarray]:
    """Dot2 values of (A*B)[rows[t], cols[t]] and their scales s_ij."""
    lib = _load()
    A, B = _f64(A), _f64(B)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    if rows.shape != cols.shape:
        raise ValueError("rows/cols differ in length")
    k = A.shape[1]
    if B.shape[0] != k:
        raise ValueError("inner dimensions differ")
    if rows.size and (rows.min() < 0 or rows.max() >= A.shape[0]
                      or cols.min() < 0 or cols.max() >= B.shape[1]):
        raise IndexError("sample index out of range")
    c = np.empty(rows.size, dtype=np.float64)
    s = np.empty(rows.size, dtype=np.float64)
    lib.oracle_sampled(k, _ptr(A), A.shape[1], _ptr(B), B.shape[1], rows.size,
                       _ptr(rows), _ptr(cols), _ptr(c), _ptr(s))
    return c, s


def matvec2(M, x) -> tuple[np.ndarray, np.ndarray]:
    """(M x by Dot2 per row, |M| |x|)."""
    lib = _load()
    M, x = _f64(M), _f64(x)
    r, c = M.shape
    y = np.empty(r, dtype=np.float64)
    sy = np.empty(r, dtype=np.float64)
    lib.oracle_matvec2(r, c, _ptr(M), c, _ptr(x), _ptr(y), _ptr(sy))
    return y, sy


def gamma(n: int) -> float:
    """gamma_n = n u / (1 - n u): the classic bound factor for an n-term
    dot product in binary64 (Higham, Accuracy and Stability, Sec. 3.1)."""
    return n * U / (1.0 - n * U)


def freivalds(A, B, C_hat, x) -> tuple[np.ndarray, np.ndarray]:
    """Residual r = |C_hat x - A (B x)| and a bound it must meet.

    If C_hat is any FP64 product whose entries satisfy the classic bound
    |c_hat - c| <= gamma_K (|A||B|), then |C_hat x - C x| is at most
    gamma_K (|A|(|B||x|)).  The oracle's own Dot2 products add a few units of
    roundoff relative to |A|(|B||x|) and |C_hat||x|, covered by the extra
    4u and 2u terms.  A dropped or duplicated panel, a wrong tile or a
    transposed operand produces a residual of order |A|(|B||x|) itself.
    """
    K = np.asarray(A).shape[1]
    x = _f64(x)
    y, sy = matvec2(B, x)          # B x and |B||x|
    z, _ = matvec2(A, y)           # A (B x)
    _, sz = matvec2(np.abs(_f64(A)), sy)  # |A| (|B||x|)
    w, sw = matvec2(C_hat, x)      # C_hat x, |C_hat||x|
    resid = np.abs(w - z)
    bound = (gamma(K) + 4 * U) * sz + 2 * U * sw
    return resid, bound


# ---------------------------------------------------------------- exact ----

def exact_product(A, B) -> np.ndarray:
    """A*B in exact rational arithmetic, each entry rounded once to binary64.

    Every binary64 value is a dyadic rational, so Fraction(a) is exact and the
    sum of products is the exact mathematical value of c_ij = sum_k a_ik b_kj;
    float(Fraction) rounds to nearest-even.  Tiny inputs only.
    """
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    m, k = A.shape
    n = B.shape[1]
    Af = [[Fraction(float(A[i, t])) for t in range(k)] for i in range(m)]
    Bf = [[Fraction(float(B[t, j])) for j in range(n)] for t in range(k)]
    C = np.empty((m, n), dtype=np.float64)
    for i in range(m):
        for j in range(n):
            acc = Fraction(0)
            for t in range(k):
                acc += Af[i][t] * Bf[t][j]
            C[i, j] = float(acc)
    return C


def python_gemm(A, B) -> np.ndarray:
    """The same k-ordered sum as gemm(), written in pure Python floats."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    m, k = A.shape
    n = B.shape[1]
    C = np.zeros((m, n), dtype=np.float64)
    for i in range(m):
        for j in range(n):
            c = 0.0
            for t in range(k):
                c = c + float(A[i, t]) * float(B[t, j])
            C[i, j] = c
    return C
