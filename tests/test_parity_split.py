"""GPU parity of the precision form (BF16 / FP8-e4m3 / INT8 digit split).

Pins, in order of strength:
  * the matrix cores accumulate integer digit products exactly while the
    partial sums stay within 2^24 (hsumma_mfma_exact_probe vs Python ints);
  * the digit planes and exponents the GPU writes equal the oracle's split
    (oracle/split_ref.py) bit for bit;
  * integer-valued operands that are one digit wide give the exact product;
  * every entry is within FP64 accumulation error of the oracle's exact
    value of the truncated split product (split_ref.truncated_entries);
  * the accuracy gate: max |c_hat - c| / (|A||B|)_ij <= 1e-14 for BF16 and
    INT8 with the per-panel slice choice (c = Dot2 oracle), also reported for
    the plain relative error.  FP8 (at most 34 bits with 7 slices) is
    reported, not gated.
"""
import sys

import numpy as np
import pytest

from oracle import core, split_ref
from paper_1306_4161_amd import hsumma as hs
from paper_1306_4161_amd import inputs

from gpu_helpers import check_freivalds, dev, host

pytestmark = pytest.mark.gpu

GATE = 1e-14


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(plan, A, B):
    import torch
    C = torch.empty((plan.m, plan.n), dtype=torch.float64, device="cuda")
    ws = plan.workspace()
    plan.run(dev(A) if isinstance(A, np.ndarray) else A,
             dev(B) if isinstance(B, np.ndarray) else B, C, ws=ws)
    return host(C), ws


def _bf16_bits(x):
    import torch
    t = torch.from_numpy(np.asarray(x, dtype=np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).numpy().astype(np.uint16)


def _e4m3_bits(x):
    import torch
    t = torch.from_numpy(np.asarray(x, dtype=np.float32)).to(torch.float8_e4m3fn)
    return t.view(torch.uint8).numpy()


# ------------------------------------------------------------- exactness --

@pytest.mark.parametrize("fmt,lim,k", [(0, 256, 256), (0, 256, 16), (1, 16, 2048), (1, 16, 48)])
def test_mfma_accumulation_exact_to_2_24(fmt, lim, k):
    import torch
    _say("case probe fmt=%d k=%d" % (fmt, k))
    r = np.random.default_rng(k + fmt)
    for trial in range(3):
        if trial == 0:   # every partial sum as large as allowed
            a = np.full((32, k), lim); b = np.full((k, 32), lim)
            a[1::2] = -lim
        else:
            a = r.integers(-lim, lim + 1, (32, k)); b = r.integers(-lim, lim + 1, (k, 32))
        bits = _bf16_bits if fmt == 0 else _e4m3_bits
        da = torch.from_numpy(np.ascontiguousarray(bits(a))).cuda()
        db = torch.from_numpy(np.ascontiguousarray(bits(b))).cuda()
        d = hs.mfma_exact_probe(fmt, da, db)
        exact = a.astype(object) @ b.astype(object)
        got = host(d).astype(np.float64)
        assert np.array_equal(got, exact.astype(np.float64)), (fmt, k, trial)
        assert np.abs(exact).max() <= 2 ** 24


@pytest.mark.parametrize("k", [32, 1024])
def test_int8_mfma_accumulation_exact_to_2_24(k):
    import torch
    _say("case probe int8 k=%d" % k)
    r = np.random.default_rng(k + 7)
    for trial in range(3):
        if trial == 0:   # products of -128 x -128 = 2^14 add up to 2^24 at k = 1024
            a = np.full((32, k), -128); b = np.full((k, 32), -128)
            a[1::2] = 127
        else:
            a = r.integers(-128, 128, (32, k)); b = r.integers(-128, 128, (k, 32))
        da = torch.from_numpy(a.astype(np.int8)).cuda()
        db = torch.from_numpy(b.astype(np.int8)).cuda()
        d = hs.mfma_exact_probe(2, da, db)
        exact = a.astype(object) @ b.astype(object)
        assert np.array_equal(host(d).astype(np.float64), exact.astype(np.float64)), (k, trial)
        assert np.abs(exact).max() <= 2 ** 24


# ------------------------------------------------------------ split stage --

@pytest.mark.parametrize("prec,fmt", [(hs.SPLIT_BF16, "bf16"), (hs.SPLIT_FP8, "e4m3"),
                                      (hs.SPLIT_INT8, "int8")])
def test_digit_planes_match_oracle_bitwise(prec, fmt):
    import torch
    _say("case split planes %s" % fmt)
    m, k, n, M = 96, 100, 80, 100
    A = inputs.exponent_spread(m, k, 3, sigma=2.0)
    B = inputs.exponent_spread(k, n, 4, sigma=2.0)
    # the digit planes at a fixed count (the automatic count may send such a
    # narrow, widely spread panel to the FP64 kernel, which writes no digits)
    p = hs.Plan(n, 2, 2, 1, 100, M, m=m, k=k, prec=prec, slices=8 if fmt == "int8" else 7)
    C, ws = _run(p, A, B)
    lay = p.split_layout()
    Wp, planes = lay["Wp"], lay["planes"]
    used = p.panel_slices(ws)[0]        # one panel (k = M); planes beyond it are not written
    assert 1 <= used <= planes
    raw = ws.cpu().numpy()
    esz = 2 if fmt == "bf16" else 1
    dt = np.uint16 if esz == 2 else np.uint8
    # planes are stored in k-blocks of the product kernel's step, [plane][k //
    # kb][row][k % kb]: kb = 16 for BF16 and FP8, 32 for INT8
    kb = 32 if fmt == "int8" else 16
    digA = raw[lay["off_digA"]: lay["off_digA"] + planes * m * Wp * esz].view(dt)
    digA = digA.reshape(planes, Wp // kb, m, kb).transpose(0, 2, 1, 3).reshape(planes, m, Wp)
    digB = raw[lay["off_digB"]: lay["off_digB"] + planes * n * Wp * esz].view(dt)
    digB = digB.reshape(planes, Wp // kb, n, kb).transpose(0, 2, 1, 3).reshape(planes, n, Wp)
    eA = raw[lay["off_eA"]: lay["off_eA"] + 4 * m].view(np.int32)
    fB = raw[lay["off_fB"]: lay["off_fB"] + 4 * n].view(np.int32)
    e_ref = split_ref.exponents(A, axis=1)
    f_ref = split_ref.exponents(B, axis=0)
    assert np.array_equal(eA, e_ref) and np.array_equal(fB, f_ref)
    # the INT8 carries depend on the count, so its digits are those of `used`
    sd = used if fmt == "int8" else planes
    DA = split_ref.digits(A, e_ref, sd, fmt, axis=1)           # (s, m, k)
    DB = split_ref.digits(B, f_ref, sd, fmt, axis=0)           # (s, k, n)
    t = split_ref.FORMATS[fmt][1]
    for l in range(used):
        if fmt == "bf16":
            wa = _bf16_bits(np.ldexp(DA[l], -t * l))
            wb = _bf16_bits(np.ldexp(DB[l].T, -t * l))
        elif fmt == "int8":
            wa = DA[l].astype(np.int8).view(np.uint8)
            wb = np.ascontiguousarray(DB[l].T).astype(np.int8).view(np.uint8)
        else:
            # a zero digit may come out as +0 or -0 (0x80); both are the value 0
            wa = _e4m3_bits(DA[l]); wa[wa == 0x80] = 0
            wb = _e4m3_bits(DB[l].T); wb[wb == 0x80] = 0
        assert np.array_equal(digA[l, :, :k], wa), l
        assert np.array_equal(digB[l, :, :k], wb), l
        assert not digA[l, :, k:].any() and not digB[l, :, k:].any()


# -------------------------------------------------------- exact products --

@pytest.mark.parametrize("prec,r", [(hs.SPLIT_BF16, 8), (hs.SPLIT_FP8, 4), (hs.SPLIT_INT8, 6)])
def test_integer_operands_one_digit_exact(prec, r):
    _say("case integer one-digit prec=%d" % prec)
    n = 320
    A = inputs.integer_valued(n, n, 71, r)
    B = inputs.integer_valued(n, n, 72, r)
    for slices in (1, 3, 0):
        p = hs.Plan(n, 2, 2, 4, 64, 128, prec=prec, slices=slices, min_slices=1)
        C, _ = _run(p, A, B)
        assert np.array_equal(C, core.gemm(A, B)), slices


def test_identity_exact_for_six_digits():
    # entries in +-[1/2, 1): six BF16 digits (8 + 5 x 9 = 53 bits) hold every
    # bit, and B = I has one digit, so the product is exact
    n = 256
    r = np.random.default_rng(81)
    A = r.uniform(0.5, 1.0, (n, n)) * r.choice([-1.0, 1.0], (n, n))
    p = hs.Plan(n, 2, 2, 1, 128, 128, prec=hs.SPLIT_BF16, slices=6)
    C, _ = _run(p, A, np.eye(n))
    assert np.array_equal(C, A)


# ---------------------------------------------- truncated product parity --

@pytest.mark.parametrize("prec,fmt,s", [(hs.SPLIT_BF16, "bf16", 4), (hs.SPLIT_BF16, "bf16", 6),
                                        (hs.SPLIT_FP8, "e4m3", 5), (hs.SPLIT_INT8, "int8", 3),
                                        (hs.SPLIT_INT8, "int8", 8)])
def test_equals_truncated_split_product(prec, fmt, s):
    _say("case truncated %s s=%d" % (fmt, s))
    m, k, n, M = 130, 300, 110, 128
    A = inputs.exponent_spread(m, k, 91, sigma=2.0)
    B = inputs.exponent_spread(k, n, 92, sigma=2.0)
    p = hs.Plan(n, 2, 2, 2, 64, M, m=m, k=k, prec=prec, slices=s, min_slices=1)
    C, _ = _run(p, A, B)
    rows, cols = np.meshgrid(np.arange(0, m, 3), np.arange(0, n, 4), indexing="ij")
    rows, cols = rows.ravel(), cols.ravel()
    T = split_ref.truncated_entries(A, B, M, s, fmt, rows, cols)
    S = (np.abs(A) @ np.abs(B))[rows, cols]
    # FP64 additions: one per level per 32..64 k plus one per panel
    nadd = 8 * (k // 32 + 2) + 4 * (k // M + 1)
    tol = nadd * core.U * (S + np.abs(T))
    assert np.all(np.abs(C[rows, cols] - T) <= tol)


def test_bf16_deep_levels_round_within_their_bound():
    # BF16 digit pairs of levels 4 and up (l1 + l2 >= 6) share one FP32
    # accumulator, which rounds; INT8 keeps every level exact.  A wide spread
    # (sigma = 3, k = 1024) with the slice count fixed, so that the panel is
    # split rather than sent to the FP64 kernel, against the oracle's exact
    # truncated product T of the same digits: INT8 within the FP64 additions'
    # bound, BF16 within that plus the deep accumulator's stated estimate
    # 2^-60.5 kappa_A kappa_B / sqrt(k) of (|A||B|)_ij (kappa = max|x| w /
    # sum|x| of the worst line), with a factor 16 of margin on the estimate
    # (measured: INT8 2.0e-16, BF16 9.5e-14 -- above the FP64 additions'
    # bound, so the deep rounding shows -- against an estimate of 1.0e-14).
    _say("case BF16 deep levels sigma=3")
    m, k, n, M = 96, 1024, 80, 1024
    A = inputs.exponent_spread(m, k, 151, sigma=3.0)
    B = inputs.exponent_spread(k, n, 152, sigma=3.0)
    rows, cols = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    rows, cols = rows.ravel()[::2], cols.ravel()[::2]
    S = (np.abs(A) @ np.abs(B))[rows, cols]
    nadd = 8 * (k // 32 + 2) + 4 * (k // M + 1)
    kA = np.max(np.max(np.abs(A), axis=1) * k / np.sum(np.abs(A), axis=1))
    kB = np.max(np.max(np.abs(B), axis=0) * k / np.sum(np.abs(B), axis=0))
    deep = 16 * 2.0 ** -60.5 * kA * kB / np.sqrt(k)
    for prec, fmt, s in ((hs.SPLIT_INT8, "int8", 8), (hs.SPLIT_BF16, "bf16", 7)):
        p = hs.Plan(n, 2, 2, 2, 64, M, m=m, k=k, prec=prec, slices=s, min_slices=1)
        C, ws = _run(p, A, B)
        assert p.panel_slices(ws) == [s]
        T = split_ref.truncated_entries(A, B, M, s, fmt, rows, cols)
        err = np.abs(C[rows, cols] - T)
        tol = nadd * core.U * (S + np.abs(T))
        _say("  %s s=%d: max |C - T| / (|A||B|) %.3g (FP64 additions' bound %.3g, deep "
             "estimate with margin %.3g)" % (fmt, s, np.max(err / S), np.max(tol / S), deep))
        if fmt == "int8":
            assert np.all(err <= tol)
        else:
            assert np.all(err <= tol + deep * S)
        p.close()


@pytest.mark.parametrize("prec,fmt,s", [(hs.SPLIT_INT8, "int8", 8), (hs.SPLIT_BF16, "bf16", 7)])
def test_truncated_product_with_many_items_per_workgroup(prec, fmt, s):
    # 2000 x 1900 with 64 x 128 macro-tiles is 32 x 15 = 480 items, so most
    # persistent workgroups run two (or more) items back to back: the INT8
    # kernel then issues an item's first DMA steps during the previous
    # item's epilogue and leaves that item's C writes in flight across its
    # first wait.  Ragged last rows and columns, two panels.
    _say("case truncated many items %s s=%d" % (fmt, s))
    m, k, n, M = 2000, 512, 1900, 256
    A = inputs.exponent_spread(m, k, 131, sigma=2.0)
    B = inputs.exponent_spread(k, n, 132, sigma=2.0)
    p = hs.Plan(n, 2, 2, 4, 64, M, m=m, k=k, prec=prec, slices=s, min_slices=1)
    assert p.num_items > 256
    C, _ = _run(p, A, B)
    r = np.random.default_rng(5)
    rows = np.concatenate([r.integers(0, m, 300), np.arange(m - 8, m), np.arange(8)])
    cols = np.concatenate([r.integers(0, n, 300), np.arange(n - 8, n), np.arange(8)])
    T = split_ref.truncated_entries(A, B, M, s, fmt, rows, cols)
    S = np.einsum("ij,ji->i", np.abs(A[rows]), np.abs(B[:, cols]))
    nadd = 8 * (k // 32 + 2) + 4 * (k // M + 1)
    tol = nadd * core.U * (S + np.abs(T))
    assert np.all(np.abs(C[rows, cols] - T) <= tol)


@pytest.mark.parametrize("prec,fmt,s", [(hs.SPLIT_INT8, "int8", 6), (hs.SPLIT_BF16, "bf16", 5)])
def test_local_updates_are_truncated_products_of_inner_panels(prec, fmt, s):
    # hsumma_local_update splits the k-range of its inner step on its own, so
    # the sum of every step's update is the truncated split product with
    # panels of width b (here with a fixed slice count)
    import torch
    _say("case local updates %s s=%d" % (fmt, s))
    m, k, n, b, M = 200, 384, 170, 64, 128
    A = inputs.exponent_spread(m, k, 141, sigma=2.0)
    B = inputs.exponent_spread(k, n, 142, sigma=2.0)
    p = hs.Plan(n, 2, 2, 2, b, M, m=m, k=k, prec=prec, slices=s, min_slices=1)
    ws = p.workspace()
    dA, dB = dev(A), dev(B)
    C = torch.zeros((m, n), dtype=torch.float64, device="cuda")
    for st in range(p.num_steps):
        p.local_update(st, dA, dB, C, ws=ws)
    C = host(C)
    rows, cols = np.meshgrid(np.arange(0, m, 3), np.arange(0, n, 2), indexing="ij")
    rows, cols = rows.ravel(), cols.ravel()
    T = split_ref.truncated_entries(A, B, b, s, fmt, rows, cols)
    S = (np.abs(A) @ np.abs(B))[rows, cols]
    nadd = 8 * (k // 32 + 2) + 4 * (k // b + 1)
    tol = nadd * core.U * (S + np.abs(T))
    assert np.all(np.abs(C[rows, cols] - T) <= tol)


# ---------------------------------------------------------- accuracy gate --

@pytest.mark.parametrize("prec", [hs.SPLIT_BF16, hs.SPLIT_INT8])
@pytest.mark.parametrize("dist", ["uniform", "spread2"])
def test_auto_slices_meet_gate(dist, prec):
    _say("case gate %s prec=%d" % (dist, prec))
    n = 1024
    if dist == "uniform":
        A = inputs.uniform(n, n, 101); B = inputs.uniform(n, n, 102)
    else:
        A = inputs.exponent_spread(n, n, 101, 2.0); B = inputs.exponent_spread(n, n, 102, 2.0)
    p = hs.Plan(n, 4, 4, 4, 256, 256, prec=prec)
    C, ws = _run(p, A, B)
    rows, cols = inputs.sample_entries(n, n, 4096, inputs.SEED_SAMPLE)
    c, s = core.sampled(A, B, rows, cols)
    err = np.abs(C[rows, cols] - c) / s
    _say("  slices per panel %r  max scaled err %.3g  max pure %.3g" % (
        p.panel_slices(ws), err.max(), np.max(np.abs(C[rows, cols] - c) / np.abs(c))))
    assert err.max() <= GATE
    check_freivalds(A, B, C, seeds=(1,))


def test_fp8_reports_error_within_truncation_bound():
    n = 512
    A = inputs.uniform(n, n, 111)
    B = inputs.uniform(n, n, 112)
    p = hs.Plan(n, 2, 2, 1, 256, 256, prec=hs.SPLIT_FP8, slices=7)
    C, _ = _run(p, A, B)
    rows, cols = inputs.sample_entries(n, n, 1024, 5)
    c, s = core.sampled(A, B, rows, cols)
    err = np.abs(C[rows, cols] - c) / s
    # 7 e4m3 digits keep 4 + 5*6 = 34 bits of each operand
    assert err.max() <= 64 * 2.0 ** -34
    _say("  fp8 s=7 max scaled err %.3g" % err.max())


@pytest.mark.parametrize("prec", [hs.SPLIT_BF16, hs.SPLIT_INT8])
def test_c2_shape_sampled(prec):
    _say("case c2 split prec=%d n=16384" % prec)
    n = 16384
    A = inputs.uniform(n, n, inputs.SEED_A)
    B = inputs.uniform(n, n, inputs.SEED_B)
    p = hs.Plan(n, 16, 16, 16, 256, 256, prec=prec)
    C, ws = _run(p, A, B)
    edges = [i * n // 16 for i in range(16)]
    rows, cols = inputs.sample_entries(n, n, 2048, inputs.SEED_SAMPLE, edges, edges, per_edge=4)
    c, s = core.sampled(A, B, rows, cols)
    err = np.abs(C[rows, cols] - c) / s
    _say("  slices %r max scaled err %.3g" % (sorted(set(p.panel_slices(ws))), err.max()))
    assert err.max() <= GATE


# ------------------------------------------------- edges and batching form --

@pytest.mark.parametrize("shape", [
    # m, k, n, P, Q, G, b, M
    (1, 1, 1, 1, 1, 1, 1, 1),
    (1, 300, 7, 1, 1, 1, 100, 300),
    (65, 17, 129, 1, 2, 2, 17, 17),
    (3, 1000, 2, 1, 1, 1, 250, 500),
    (200, 64, 1, 2, 1, 2, 64, 64),
    (96, 2, 96, 1, 1, 1, 2, 2),
    (96, 33, 96, 1, 1, 1, 33, 33),
])
@pytest.mark.parametrize("prec", [hs.SPLIT_BF16, hs.SPLIT_INT8])
def test_degenerate_shapes_meet_gate(shape, prec):
    # exponent-spread entries on narrow panels: the per-line spread statistic
    # saturates at the panel width there, and the slice choice must still
    # meet the gate
    m, k, n, P, Q, G, b, M = shape
    _say("case split degenerate %r prec=%d" % (shape, prec))
    A = inputs.exponent_spread(m, k, 121, 2.0)
    B = inputs.exponent_spread(k, n, 122, 2.0)
    p = hs.Plan(n, P, Q, G, b, M, m=m, k=k, prec=prec)
    C, ws = _run(p, A, B)
    rows, cols = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    rows, cols = rows.ravel(), cols.ravel()
    c, s = core.sampled(A, B, rows, cols)
    err = np.abs(C[rows, cols] - c) / np.where(s > 0, s, 1.0)
    slices = p.panel_slices(ws)
    _say("  slices %r max scaled err %.3g" % (slices, err.max()))
    # 0: the panel went to the FP64 kernel
    assert all(x == 0 or 3 <= x <= (8 if prec == hs.SPLIT_INT8 else 7) for x in slices)
    assert err.max() <= GATE


@pytest.mark.parametrize("prec", [hs.SPLIT_BF16, hs.SPLIT_INT8])
def test_c3_block_cyclic_split_graph(prec):
    import torch
    _say("case c3 split prec=%d: n=10000 6x10 block-cyclic b=128 persistent+graph" % prec)
    n = 10000
    A = inputs.uniform(n, n, inputs.SEED_A)
    B = inputs.uniform(n, n, inputs.SEED_B)
    p = hs.Plan(n, 6, 10, 1, 128, dist=hs.DIST_BLOCK_CYCLIC, prec=prec,
                persistent=1, use_graph=1)
    ws = p.workspace()
    dA, dB = dev(A), dev(B)
    C = torch.empty((n, n), dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()
    outs = []
    for rep in range(3):
        stream.wait_stream(torch.cuda.current_stream())  # after the eager work
        with torch.cuda.stream(stream):
            C.fill_(float("nan"))
            ws.fill_(0xA5)  # the graph regenerates the work-item table on each replay
            p.run(dA, dB, C, ws=ws, stream=stream)
        stream.synchronize()
        outs.append(host(C))
        dA.add_(0.0)  # eager work between replays
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    Cn = outs[0]
    edges = list(range(0, n, 128))
    rows, cols = inputs.sample_entries(n, n, 2048, inputs.SEED_SAMPLE, edges, edges, per_edge=2)
    c, s = core.sampled(A, B, rows, cols)
    err = np.abs(Cn[rows, cols] - c) / s
    _say("  slices %r max scaled err %.3g" % (sorted(set(p.panel_slices(ws))), err.max()))
    assert err.max() <= GATE
    check_freivalds(A, B, Cn)
    # the launch without the graph gives the same bits
    q = hs.Plan(n, 6, 10, 1, 128, dist=hs.DIST_BLOCK_CYCLIC, prec=prec)
    assert np.array_equal(_run(q, dA, dB)[0], Cn)


# ------------------------------------------------------- the FP64 route --
# A panel the split cannot carry to FP64 accuracy goes to the FP64 kernel
# (slice count 0): a non-finite value in the panel, or a modelled need above
# max_slices digits.  The FP64 kernel's sums do not depend on the
# macro-tile, so such a panel gives the FP64 path's bits.

def _fp64_reference(n, P, Q, G, b, M, A, B, **kw):
    import torch
    p = hs.Plan(n, P, Q, G, b, M, **kw)
    C = torch.empty((p.m, p.n), dtype=torch.float64, device="cuda")
    p.run(A, B, C, ws=p.workspace())
    return host(C)


@pytest.mark.parametrize("prec", [hs.SPLIT_BF16, hs.SPLIT_INT8, hs.SPLIT_FP8])
def test_need_beyond_max_slices_takes_fp64_route(prec):
    _say("case route: need beyond max_slices prec=%d" % prec)
    n, P, Q, G, b, M = 512, 2, 2, 4, 64, 256
    A = dev(inputs.exponent_spread(n, n, 131, 2.0))
    B = dev(inputs.exponent_spread(n, n, 132, 2.0))
    p = hs.Plan(n, P, Q, G, b, M, prec=prec, max_slices=3)   # 3 digits never suffice
    C, ws = _run(p, A, B)
    assert p.panel_slices(ws) == [0, 0]
    assert np.array_equal(C, _fp64_reference(n, P, Q, G, b, M, A, B))


@pytest.mark.parametrize("prec", [hs.SPLIT_BF16, hs.SPLIT_INT8])
def test_nonfinite_values_take_fp64_route(prec):
    import torch
    _say("case route: non-finite prec=%d" % prec)
    n, P, Q, G, b, M = 384, 3, 2, 6, 32, 128
    A = inputs.uniform(n, n, 141)
    B = inputs.uniform(n, n, 142)
    A[5, 10] = np.nan                # panel 0
    B[300, 7] = np.inf               # panel 2
    A[200, 301] = -np.inf            # panel 2
    dA, dB = dev(A), dev(B)
    p = hs.Plan(n, P, Q, G, b, M, prec=prec)
    C, ws = _run(p, dA, dB)
    sl = p.panel_slices(ws)
    assert sl[0] == 0 and sl[2] == 0 and sl[1] > 0
    ref = _fp64_reference(n, P, Q, G, b, M, dA, dB)
    # every non-finite entry of the FP64 product is the same non-finite
    # value here: row 5 NaN, column 7 +-Inf or NaN, row 200 -Inf or NaN
    bad = ~np.isfinite(ref)
    assert bad[5].all() and bad[:, 7].all() and bad[200].all()
    assert np.array_equal(np.isnan(C), np.isnan(ref))
    assert np.array_equal(C[bad & ~np.isnan(ref)], ref[bad & ~np.isnan(ref)])
    # the finite entries meet the gate
    good = np.argwhere(~bad)[::97]
    rows, cols = good[:, 0], good[:, 1]
    c, s = core.sampled(A, B, rows, cols)
    assert np.max(np.abs(C[rows, cols] - c) / s) <= GATE
    # with every panel holding a NaN the whole product is the FP64 path's
    A2 = A.copy()
    A2[0, ::M] = np.nan
    dA2 = dev(A2)
    C2, ws2 = _run(p, dA2, dB)
    assert p.panel_slices(ws2) == [0, 0, 0]
    ref2 = _fp64_reference(n, P, Q, G, b, M, dA2, dB)
    assert np.array_equal(np.isnan(C2), np.isnan(ref2))
    fin = np.isfinite(ref2)
    assert np.array_equal(C2[fin], ref2[fin])


@pytest.mark.parametrize("prec", [hs.SPLIT_BF16, hs.SPLIT_INT8])
@pytest.mark.parametrize("kind", ["third", "tenth", "signed_third_gram"])
@pytest.mark.parametrize("k", [1024, 4096])
def test_repeated_magnitudes_meet_gate(kind, prec, k):
    # Lines of one repeated magnitude: the digits' truncation errors of every
    # term have the same sign, so no cancellation over k may be credited.
    _say("case repeated magnitudes %s prec=%d k=%d" % (kind, prec, k))
    m = n = 256
    if kind == "third":
        A = np.full((m, k), 1.0 / 3.0); B = np.full((k, n), 1.0 / 3.0)
    elif kind == "tenth":
        A = np.full((m, k), 0.1); B = np.full((k, n), 0.1)
    else:
        # C = S S^T with S = +-1/3: the diagonal sums k equal products
        S = np.where(inputs.rademacher(m * k, 151).reshape(m, k) > 0, 1.0, -1.0) / 3.0
        A = S; B = np.ascontiguousarray(S.T[:, :n])
    p = hs.Plan(n, 2, 2, 1, 256, 256, m=m, k=k, prec=prec)
    C, ws = _run(p, A, B)
    rows, cols = np.meshgrid(np.arange(0, m, 7), np.arange(0, n, 5), indexing="ij")
    rows, cols = np.concatenate([rows.ravel(), np.arange(n)]), np.concatenate([cols.ravel(), np.arange(n)])
    c, s = core.sampled(A, B, rows, cols)
    err = np.abs(C[rows, cols] - c) / s
    _say("  slices %r max scaled err %.3g" % (sorted(set(p.panel_slices(ws))), err.max()))
    assert err.max() <= GATE


@pytest.mark.parametrize("prec", [hs.SPLIT_BF16, hs.SPLIT_INT8])
@pytest.mark.parametrize("sigma,k", [(2.0, 4096), (2.5, 1024), (2.5, 4096), (3.0, 64),
                                     (3.0, 256), (3.0, 1024), (3.0, 4096), (4.0, 1024)])
def test_wide_spreads_meet_gate(sigma, k, prec):
    # Exponent spreads beyond sigma = 2 saturate the arithmetic spread
    # statistic on every panel; the geometric one decides between the
    # largest slice count and the FP64 route, and every entry meets the gate.
    _say("case wide spread sigma=%g k=%d prec=%d" % (sigma, k, prec))
    m = n = 96
    M = min(k, 1024)
    A = inputs.exponent_spread(m, k, 121 + k, sigma)
    B = inputs.exponent_spread(k, n, 122 + k, sigma)
    p = hs.Plan(n, 1, 1, 1, M, M, m=m, k=k, prec=prec)
    C, ws = _run(p, A, B)
    rows, cols = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    rows, cols = rows.ravel(), cols.ravel()
    c, s = core.sampled(A, B, rows, cols)
    err = np.abs(C[rows, cols] - c) / s
    _say("  slices %r max scaled err %.3g" % (p.panel_slices(ws), err.max()))
    assert err.max() <= GATE


@pytest.mark.parametrize("prec", [hs.SPLIT_BF16, hs.SPLIT_INT8])
def test_sigma3_at_n4096_meets_gate(prec):
    _say("case sigma=3 n=4096 prec=%d" % prec)
    n = 4096
    A = inputs.exponent_spread(n, n, inputs.SEED_A, 3.0)
    B = inputs.exponent_spread(n, n, inputs.SEED_B, 3.0)
    p = hs.Plan(n, 4, 4, 4, 256, 1024, prec=prec)
    C, ws = _run(p, A, B)
    edges = [i * n // 4 for i in range(4)]
    rows, cols = inputs.sample_entries(n, n, 2048, inputs.SEED_SAMPLE, edges, edges, per_edge=8)
    c, s = core.sampled(A, B, rows, cols)
    err = np.abs(C[rows, cols] - c) / s
    _say("  slices %r max scaled err %.3g" % (p.panel_slices(ws), err.max()))
    assert err.max() <= GATE
    check_freivalds(A, B, C, seeds=(1,))
