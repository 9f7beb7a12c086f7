"""GPU parity of the FP64 MFMA local update against the CPU oracle.

Tolerance: each entry of an FP64 product of inner length K may differ from
the exact value by gamma_K (|A||B|)_ij (the classic dot-product bound,
valid for any summation order); the reference is Dot2 (about twice working
precision), whose own error adds u|c|.  Exact cases (identity, diagonal,
rank-1, integer-valued operands) are compared bit for bit, and so are
results that the method makes independent of the schedule: the sum of the
panel updates does not depend on G, on the P x Q decomposition or on the
macro-tile, and hsumma_run equals its sequence of hsumma_local_update calls.
"""
import sys

import numpy as np
import pytest

from oracle import core
from paper_1306_4161_amd import hsumma as hs
from paper_1306_4161_amd import inputs

from gpu_helpers import check_freivalds, check_sampled, dev, host

pytestmark = pytest.mark.gpu


def _run(plan, A, B, **kw):
    import torch
    C = torch.empty((plan.m, plan.n), dtype=torch.float64, device="cuda")
    kw.setdefault("ws", plan.workspace())
    plan.run(dev(A) if isinstance(A, np.ndarray) else A,
             dev(B) if isinstance(B, np.ndarray) else B, C, **kw)
    return host(C)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_c0_plain_summa_full_compare():
    _say("case c0: n=256 2x2 G=1 b=32")
    n = 256
    A = inputs.uniform(n, n, inputs.SEED_A)
    B = inputs.uniform(n, n, inputs.SEED_B)
    p = hs.Plan(n, 2, 2, 1, 32)
    assert p.num_steps == 8
    C = _run(p, A, B)
    rows, cols = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    check_sampled(A, B, C, rows.ravel(), cols.ravel())
    # 32 x 32 corner against exact rational arithmetic
    E = core.exact_product(A[:32], B[:, :32])
    S = np.abs(A[:32]) @ np.abs(B[:, :32])
    assert np.all(np.abs(C[:32, :32] - E) <= core.gamma(n) * S)


@pytest.mark.parametrize("shape", [
    # m, k, n, P, Q, G, b, M
    (300, 173, 257, 3, 2, 2, 24, 48),
    (129, 65, 127, 1, 1, 1, 5, 10),
    (64, 1, 64, 2, 2, 4, 1, 1),
    (17, 300, 9, 1, 1, 1, 300, 300),
    (520, 520, 520, 5, 4, 20, 52, 104),
])
def test_ragged_shapes_full_compare(shape):
    m, k, n, P, Q, G, b, M = shape
    _say("case ragged %r" % (shape,))
    A = inputs.uniform(m, k, 11)
    B = inputs.uniform(k, n, 12)
    p = hs.Plan(n, P, Q, G, b, M, m=m, k=k)
    C = _run(p, A, B)
    rows, cols = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    check_sampled(A, B, C, rows.ravel(), cols.ravel())


def test_run_equals_local_updates_and_outer_updates_bitwise():
    import torch
    _say("case run-vs-steps n=384 3x3 G=3 b=16 M=64")
    n = 384
    A = inputs.uniform(n, n, 21)
    B = inputs.uniform(n, n, 22)
    p = hs.Plan(n, 3, 3, 3, 16, 64)
    Cr = _run(p, A, B)
    dA, dB = dev(A), dev(B)
    ws = p.workspace()
    C1 = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    for s in range(p.num_steps):
        p.local_update(s, dA, dB, C1, ws=ws)
    C2 = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    for g in range(p.num_outer_steps):
        p.outer_update(g, dA, dB, C2, ws=ws)
    assert np.array_equal(host(C1), Cr)
    assert np.array_equal(host(C2), Cr)


def test_prefix_invariant_after_each_step():
    import torch
    _say("case prefix n=200 b=24")
    n = 200
    A = inputs.uniform(n, n, 31)
    B = inputs.uniform(n, n, 32)
    p = hs.Plan(n, 2, 4, 2, 24, 48)
    dA, dB = dev(A), dev(B)
    ws = p.workspace()
    C = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    rows, cols = np.meshgrid(np.arange(0, n, 3), np.arange(0, n, 5), indexing="ij")
    rows, cols = rows.ravel(), cols.ravel()
    for s in range(p.num_steps):
        p.local_update(s, dA, dB, C, ws=ws)
        e = p.step_info(s)["k1"]
        check_sampled(A[:, :e], B[:e, :], host(C), rows, cols)


def test_schedule_invariance_bitwise():
    _say("case invariance n=512")
    n = 512
    A = inputs.uniform(n, n, 41)
    B = inputs.uniform(n, n, 42)
    ref = _run(hs.Plan(n, 1, 1, 1, 32, 32), A, B)
    configs = [
        dict(P=2, Q=2, G=1, M=32), dict(P=2, Q=2, G=4, M=32), dict(P=4, Q=4, G=4, M=128),
        dict(P=2, Q=8, G=16, M=64), dict(P=8, Q=2, G=2, M=512), dict(P=4, Q=4, G=16, M=256),
    ]
    for c in configs:
        p = hs.Plan(n, c["P"], c["Q"], c["G"], 32, c["M"])
        assert np.array_equal(_run(p, A, B), ref), c
    for tm, tn, kc, w in [(128, 128, 16, 0), (128, 128, 32, 0), (64, 64, 32, 0),
                          (128, 64, 16, 0), (64, 128, 16, 0), (32, 32, 16, 0),
                          (256, 128, 16, 0), (256, 128, 8, 0), (128, 128, 16, 8),
                          (128, 256, 16, 0), (64, 256, 16, 0), (256, 64, 16, 0)]:
        p = hs.Plan(n, 4, 4, 4, 32, 64, tile_m=tm, tile_n=tn, kc=kc, waves=w)
        assert np.array_equal(_run(p, A, B), ref), (tm, tn, kc, w)
        # 1 x 2 grid: 512 x 256 tiles, so every macro-tile is full
        p = hs.Plan(n, 1, 2, 1, 32, 64, tile_m=tm, tile_n=tn, kc=kc, waves=w)
        assert np.array_equal(_run(p, A, B), ref), ("full", tm, tn, kc, w)
        # the register-staged kernel of the same configuration
        p = hs.Plan(n, 2, 2, 1, 32, 64, tile_m=tm, tile_n=tn, kc=kc, waves=w, staged=1)
        assert np.array_equal(_run(p, A, B), ref), ("staged", tm, tn, kc, w)
    p = hs.Plan(n, 4, 4, 4, 32, 64, persistent=1)
    assert np.array_equal(_run(p, A, B), ref)
    p = hs.Plan(n, 4, 4, 4, 32, 64, persistent=1, wgs_per_cu=1)
    assert np.array_equal(_run(p, A, B), ref)
    p = hs.Plan(n, 4, 4, 4, 32, 64, dist=hs.DIST_BLOCK_CYCLIC, nb=64)
    assert np.array_equal(_run(p, A, B), ref)


def test_determinism_run_to_run():
    n = 1024
    A = inputs.uniform(n, n, 51)
    B = inputs.uniform(n, n, 52)
    p = hs.Plan(n, 4, 4, 4, 64, 256)
    a = _run(p, A, B)
    for _ in range(3):
        assert np.array_equal(_run(p, A, B), a)


def test_exact_special_cases_bitwise():
    _say("case special n=448")
    n = 448
    r = np.random.default_rng(5)
    A = inputs.uniform(n, n, 61)
    p = hs.Plan(n, 4, 2, 2, 64, 128)
    assert np.array_equal(_run(p, A, np.eye(n)), A)
    d = r.uniform(-2, 2, n)
    assert np.array_equal(_run(p, A, np.diag(d)), A * d[None, :])
    a = np.zeros((n, n)); a[:, 0] = r.uniform(-1, 1, n)
    b = np.zeros((n, n)); b[0, :] = r.uniform(-1, 1, n)
    assert np.array_equal(_run(p, a, b), np.outer(a[:, 0], b[0, :]))
    Ai = inputs.integer_valued(n, n, 62, 3)
    Bi = inputs.integer_valued(n, n, 63, 3)
    assert np.array_equal(_run(p, Ai, Bi), core.gemm(Ai, Bi))


def test_c1_hsumma_8192_sampled_and_freivalds():
    _say("case c1: n=8192 8x8 G=4 M=256 b=64")
    n = 8192
    A = inputs.uniform(n, n, inputs.SEED_A)
    B = inputs.uniform(n, n, inputs.SEED_B)
    p = hs.Plan(n, 8, 8, 4, 64, 256)
    assert p.groups == (2, 2) and p.num_steps == 128 and p.num_outer_steps == 32
    C = _run(p, A, B)
    edges = [i * n // 8 for i in range(8)]
    rows, cols = inputs.sample_entries(n, n, 2048, inputs.SEED_SAMPLE, edges, edges, per_edge=16)
    check_sampled(A, B, C, rows, cols)
    check_freivalds(A, B, C)


def test_c3_block_cyclic_persistent_graph():
    import torch
    _say("case c3: n=10000 6x10 block-cyclic b=128 persistent+graph")
    n = 10000
    A = inputs.uniform(n, n, inputs.SEED_A)
    B = inputs.uniform(n, n, inputs.SEED_B)
    p = hs.Plan(n, 6, 10, 1, 128, dist=hs.DIST_BLOCK_CYCLIC, persistent=1, use_graph=1)
    dA, dB = dev(A), dev(B)
    ws = p.workspace()
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
    rowedges = [g for g in range(0, n, 128)]
    rows, cols = inputs.sample_entries(n, n, 2048, inputs.SEED_SAMPLE, rowedges, rowedges,
                                       per_edge=2)
    check_sampled(A, B, Cn, rows, cols)
    check_freivalds(A, B, Cn)
    # the direct (non-graph, non-persistent) launch gives the same bits
    q = hs.Plan(n, 6, 10, 1, 128, dist=hs.DIST_BLOCK_CYCLIC)
    assert np.array_equal(_run(q, dA, dB), Cn)


@pytest.mark.parametrize("prec", [hs.FP64, hs.SPLIT_BF16, hs.SPLIT_INT8])
def test_checkpoint_resume_bitwise(prec):
    # the step boundary is a checkpoint: C after outer step s is the product
    # over the first s panels; a new plan can resume from it
    import torch
    _say("case checkpoint/resume prec=%d" % prec)
    n, P, Q, G, b, M = 768, 3, 4, 6, 32, 128
    A = dev(inputs.uniform(n, n, 71))
    B = dev(inputs.uniform(n, n, 72))
    p = hs.Plan(n, P, Q, G, b, M, prec=prec)
    ws = p.workspace()
    ref = torch.empty((n, n), dtype=torch.float64, device="cuda")
    p.run(A, B, ref, ws=ws)
    again = torch.empty_like(ref)
    p.run(A, B, again, ws=ws)
    assert torch.equal(ref, again)                       # run-to-run determinism
    nout = p.num_outer_steps
    p.close()
    C = torch.zeros_like(ref)
    first = hs.Plan(n, P, Q, G, b, M, prec=prec)
    ws1 = first.workspace()
    for g in range(nout // 2):
        first.outer_update(g, A, B, C, ws=ws1)
    torch.cuda.synchronize()
    first.close()
    del ws1
    second = hs.Plan(n, P, Q, G, b, M, prec=prec)
    ws2 = second.workspace()
    for g in range(nout // 2, nout):
        second.outer_update(g, A, B, C, ws=ws2)
    torch.cuda.synchronize()
    second.close()
    assert torch.equal(C, ref)
