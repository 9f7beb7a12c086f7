"""GPU parity of the LU factorisation whose trailing update is the HSUMMA
local update (hsumma_lu) against the LU oracle (oracle/lu_ref.py).

  * integer factors with power-of-two pivots: every partial Schur
    complement is exact, so the factors must come back bit for bit;
  * diagonally dominant matrices: the factors within a few units of the
    oracle's (relative to |L||U|), and the backward error |L U - A| within
    gamma_n |L||U| (Higham, Thm. 9.3) on every entry / on sampled entries;
  * the same with the trailing updates in the INT8 digit split.
"""
import sys

import numpy as np
import pytest

from oracle import core, lu_ref
from paper_1306_4161_amd import hsumma as hs
from paper_1306_4161_amd import inputs

from gpu_helpers import dev, host
from test_lu_ref import _integer_factors

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _factor(A, P, Q, G, b, M, **kw):
    plan = hs.LuPlan(A.shape[0], P, Q, G, b, M, **kw)
    dA = dev(A)
    plan.factor(dA, plan.workspace())
    out = host(dA)
    plan.close()
    return out


def _dominant(n, seed):
    A = inputs.uniform(n, n, seed)
    return A + np.diag(np.abs(A).sum(axis=1) + 1.0)


@pytest.mark.parametrize("n,P,Q,G,b,M", [(256, 1, 1, 1, 32, 64), (300, 2, 2, 4, 64, 128),
                                         (257, 3, 2, 6, 16, 48), (130, 2, 2, 1, 64, 64)])
def test_integer_factors_bitwise(n, P, Q, G, b, M):
    _say("case lu integer n=%d grid %dx%d G=%d b=%d M=%d" % (n, P, Q, G, b, M))
    L0, U0 = _integer_factors(n, 200 + n)
    LU = _factor(L0 @ U0, P, Q, G, b, M)
    L, U = lu_ref.unpack(LU)
    assert np.array_equal(L, L0) and np.array_equal(U, U0)


@pytest.mark.parametrize("n,P,Q,G,b,M", [(512, 2, 2, 4, 64, 256), (777, 3, 3, 9, 32, 96)])
def test_dominant_against_oracle_and_backward_error(n, P, Q, G, b, M):
    _say("case lu dominant n=%d" % n)
    A = _dominant(n, 300 + n)
    LU = _factor(A, P, Q, G, b, M)
    ref = lu_ref.lu_nopivot(A)
    L, U = lu_ref.unpack(LU)
    Lr, Ur = lu_ref.unpack(ref)
    # the factors: both are n-step eliminations of the same matrix, each
    # within gamma_n |L||U| of A; for this well-conditioned matrix they agree
    # to a few multiples of that
    scale = np.abs(Lr) @ np.abs(Ur)
    assert np.all(np.abs(L @ U - Lr @ Ur) <= 4 * core.gamma(n) * scale + 1e-300)
    assert np.max(np.abs(L - Lr)) <= 1e-13 and np.max(np.abs(U - Ur) / np.abs(np.diag(Ur))[:, None]) <= 1e-13
    rows, cols = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    rows, cols = rows.ravel(), cols.ravel()
    r, s = lu_ref.residual_sampled(LU, A, rows, cols)
    assert np.all(r <= core.gamma(n) * s + 2 * core.U * np.abs(A[rows, cols]))


@pytest.mark.parametrize("prec", [hs.FP64, hs.SPLIT_INT8])
def test_n4096_on_a_grid_sampled_backward_error(prec):
    _say("case lu n=4096 4x4 G=4 b=64 M=512 prec=%d" % prec)
    n = 4096
    A = _dominant(n, 401)
    LU = _factor(A, 4, 4, 4, 64, 512, prec=prec)
    rows, cols = inputs.sample_entries(n, n, 4096, inputs.SEED_SAMPLE,
                                       range(0, n, 512), range(0, n, 512), per_edge=4)
    r, s = lu_ref.residual_sampled(LU, A, rows, cols)
    bound = core.gamma(n) * s + 2 * core.U * np.abs(A[rows, cols])
    if prec != hs.FP64:
        # each of the n/M - 1 trailing updates adds at most 1e-14 (|L||U|)_ij
        bound = bound + (n // 512) * 1e-14 * s
    _say("  max |LU - A| / (|L||U|) = %.3g" % float(np.max(r / s)))
    assert np.all(r <= bound)
    # a row and a column of the factors against the oracle's elimination of
    # the leading 1024 x 1024 block (its factors are the leading block's)
    ref = lu_ref.lu_nopivot(A[:1024, :1024])
    assert np.max(np.abs(LU[:1024, :1024] - ref) / (np.abs(ref) + 1.0)) <= 1e-12


@pytest.mark.parametrize("n,P,Q,G,b,M", [(256, 1, 1, 1, 32, 64), (300, 2, 2, 4, 64, 128),
                                         (257, 3, 2, 6, 16, 48), (130, 2, 2, 1, 64, 64),
                                         (64, 1, 1, 1, 64, 64), (2100, 4, 4, 4, 64, 512)])
def test_lookahead_same_bits_as_plain(n, P, Q, G, b, M):
    # the look-ahead schedule splits each trailing update into three blocks
    # of the same C += (-L21) U12 with the same k order per entry: in FP64
    # the factors are the same bits, and the integer factors stay exact
    _say("case lu look-ahead n=%d grid %dx%d G=%d b=%d M=%d" % (n, P, Q, G, b, M))
    A = _dominant(n, 500 + n)
    plain = _factor(A, P, Q, G, b, M)
    ahead = _factor(A, P, Q, G, b, M, lookahead=1)
    assert np.array_equal(plain, ahead)
    L0, U0 = _integer_factors(n, 200 + n)
    L, U = lu_ref.unpack(_factor(L0 @ U0, P, Q, G, b, M, lookahead=1))
    assert np.array_equal(L, L0) and np.array_equal(U, U0)


def test_lookahead_plan_reused_and_split_form():
    import torch
    _say("case lu look-ahead reuse n=1536 int8")
    n = 1536
    A = _dominant(n, 611)
    plan = hs.LuPlan(n, 2, 2, 4, 64, 256, lookahead=1)
    ws = plan.workspace()
    outs = []
    for rep in range(2):
        ws.fill_(0x5A + rep)
        dA = dev(A)
        plan.factor(dA, ws)
        outs.append(host(dA))
    plan.close()
    assert np.array_equal(outs[0], outs[1])
    # the split form: each block of the trailing update takes its own slice
    # count, so the bits may differ from the plain schedule; both are within
    # the backward-error bound of the split
    LU = _factor(A, 2, 2, 4, 64, 256, prec=hs.SPLIT_INT8, lookahead=1)
    rows, cols = inputs.sample_entries(n, n, 2048, inputs.SEED_SAMPLE,
                                       range(0, n, 256), range(0, n, 256), per_edge=4)
    r, s = lu_ref.residual_sampled(LU, A, rows, cols)
    bound = core.gamma(n) * s + 2 * core.U * np.abs(A[rows, cols]) + (n // 256) * 1e-14 * s
    assert np.all(r <= bound)
    torch.cuda.synchronize()


def test_random_lu_plans():
    # random sizes, block sizes, grids, groupings and schedules (hypothesis):
    # integer factors with power-of-two pivots come back bit for bit, and a
    # diagonally dominant matrix's factors meet the backward-error bound on
    # every entry
    from hypothesis import given, settings, strategies as st, HealthCheck

    @st.composite
    def cases(draw):
        n = draw(st.integers(1, 300))
        b = draw(st.integers(1, 64))
        M = b * draw(st.integers(1, 4))
        P = draw(st.integers(1, 4))
        Q = draw(st.integers(1, 4))
        G = draw(st.sampled_from(sorted({I * J for I in range(1, P + 1) if P % I == 0
                                         for J in range(1, Q + 1) if Q % J == 0})))
        return n, P, Q, G, b, M, draw(st.integers(0, 1)), draw(st.integers(0, 10 ** 6))

    @settings(max_examples=50, deadline=None, suppress_health_check=[HealthCheck.too_slow])
    @given(cases())
    def check(c):
        n, P, Q, G, b, M, la, seed = c
        _say("case random lu %r" % (c,))
        L0, U0 = _integer_factors(n, seed)
        L, U = lu_ref.unpack(_factor(L0 @ U0, P, Q, G, b, M, lookahead=la))
        assert np.array_equal(L, L0) and np.array_equal(U, U0)
        A = _dominant(n, seed + 1)
        LU = _factor(A, P, Q, G, b, M, lookahead=la)
        rows, cols = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        rows, cols = rows.ravel(), cols.ravel()
        r, s = lu_ref.residual_sampled(LU, A, rows, cols)
        assert np.all(r <= core.gamma(n) * s + 2 * core.U * np.abs(A[rows, cols]))

    check()
