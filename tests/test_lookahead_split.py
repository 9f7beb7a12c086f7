"""Look-ahead of the split forms (Sec. VI: the next step's panel work
overlaps this step's update): hsumma_run with opts.lookahead splits outer
panel g + 1 on a second stream, into the other set of digit planes, while the
products of panel g run.  The kernels and their inputs are those of the plain
sequence, so the result must equal the plain run bit for bit; one case is
also held to the accuracy gate against the oracle's Dot2.
"""
import sys

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

from oracle import core
from paper_1306_4161_amd import hsumma as hs
from paper_1306_4161_amd import inputs

from gpu_helpers import dev, host
from test_items_random import plans

pytestmark = pytest.mark.gpu

GATE = 1e-14
SPLITS = [hs.SPLIT_BF16, hs.SPLIT_FP8, hs.SPLIT_INT8]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pair(n, P, Q, G, b, M, prec, **kw):
    plain = hs.Plan(n, P, Q, G, b, M, prec=prec, **kw)
    ahead = hs.Plan(n, P, Q, G, b, M, prec=prec, lookahead=1, **kw)
    return plain, ahead


def _run(plan, dA, dB, ws=None):
    import torch
    C = torch.full((plan.m, plan.n), float("nan"), dtype=torch.float64, device="cuda")
    ws = plan.workspace() if ws is None else ws
    plan.run(dA, dB, C, ws=ws)
    return C, ws


def _opts(prec):
    # FP8 reaches at most 34 bits: fixed slices keep it off the FP64 route
    return {"slices": 7} if prec == hs.SPLIT_FP8 else {}


@pytest.mark.parametrize("prec", SPLITS)
@pytest.mark.parametrize("shape", [
    (768, 3, 4, 6, 32, 128, 768),      # 6 panels
    (640, 2, 2, 4, 64, 256, 700),      # ragged last panel (k = 700)
    (512, 2, 2, 2, 64, 128, 256),      # 2 panels: one split on the second stream
    (300, 3, 2, 2, 16, 64, 1000),      # many narrow panels, ragged tiles
])
def test_lookahead_equals_plain_bitwise(prec, shape):
    import torch
    n, P, Q, G, b, M, k = shape
    _say("case lookahead prec=%d n=%d k=%d M=%d" % (prec, n, k, M))
    A = dev(inputs.exponent_spread(n, k, 11, 2.0))
    B = dev(inputs.exponent_spread(k, n, 12, 2.0))
    plain, ahead = _pair(n, P, Q, G, b, M, prec, k=k, **_opts(prec))
    assert ahead.workspace_size > plain.workspace_size
    ref, ws0 = _run(plain, A, B)
    got, ws1 = _run(ahead, A, B)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    assert plain.panel_slices(ws0) == ahead.panel_slices(ws1)
    plain.close()
    ahead.close()


def test_lookahead_meets_gate_and_reuses_plan():
    # two calls in a row on one plan (new operands, the same workspace), each
    # equal to the plain run; the second also against the oracle's Dot2
    import torch
    n, P, Q, G, b, M = 1024, 4, 4, 4, 64, 256
    _say("case lookahead reuse + gate n=%d INT8" % n)
    plain, ahead = _pair(n, P, Q, G, b, M, hs.SPLIT_INT8)
    ws = ahead.workspace()
    for seed in (21, 31):
        A = inputs.exponent_spread(n, n, seed, 2.0)
        B = inputs.exponent_spread(n, n, seed + 1, 2.0)
        dA, dB = dev(A), dev(B)
        ref, _ = _run(plain, dA, dB)
        got, _ = _run(ahead, dA, dB, ws=ws)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
    rows, cols = inputs.sample_entries(n, n, 1024, inputs.SEED_SAMPLE,
                                       list(range(0, n, 128)), list(range(0, n, 128)))
    c, s = core.sampled(A, B, rows, cols)
    err = np.abs(host(got)[rows, cols] - c) / s
    _say("  max scaled err %.3g" % err.max())
    assert err.max() <= GATE
    plain.close()
    ahead.close()


@pytest.mark.parametrize("prec", [hs.SPLIT_BF16, hs.SPLIT_INT8])
def test_lookahead_fp64_route_panel(prec):
    # an Inf in panel 1 sends that panel to the FP64 kernel (slice count 0)
    # while its neighbours are split on the second stream
    import torch
    n, P, Q, G, b, M = 512, 2, 2, 4, 32, 128
    _say("case lookahead FP64 route prec=%d" % prec)
    A = inputs.uniform(n, n, 41)
    B = inputs.uniform(n, n, 42)
    A[7, 130] = np.inf
    plain, ahead = _pair(n, P, Q, G, b, M, prec)
    ref, ws0 = _run(plain, dev(A), dev(B))
    got, ws1 = _run(ahead, dev(A), dev(B))
    torch.cuda.synchronize()
    sl = ahead.panel_slices(ws1)
    assert sl[1] == 0 and all(x > 0 for i, x in enumerate(sl) if i != 1)
    assert sl == plain.panel_slices(ws0)
    # row 7 of C is infinite in both; compare bit patterns
    assert torch.equal(got.view(torch.int64), ref.view(torch.int64))
    plain.close()
    ahead.close()


def test_lookahead_graph_replays():
    import torch
    n, P, Q, G, b, M = 768, 3, 4, 6, 32, 128
    _say("case lookahead + graph n=%d INT8" % n)
    A = dev(inputs.exponent_spread(n, n, 51, 2.0))
    B = dev(inputs.exponent_spread(n, n, 52, 2.0))
    plain = hs.Plan(n, P, Q, G, b, M, prec=hs.SPLIT_INT8)
    ref, _ = _run(plain, A, B)
    graph = hs.Plan(n, P, Q, G, b, M, prec=hs.SPLIT_INT8, lookahead=1, use_graph=1)
    ws = graph.workspace()
    C = torch.empty_like(ref)
    stream = torch.cuda.Stream()
    for rep in range(3):
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            C.fill_(float("nan"))
            ws.fill_(0x3C + rep)
            graph.run(A, B, C, ws=ws, stream=stream)
        stream.synchronize()
        assert torch.equal(C, ref)
        A.add_(0.0)
    torch.cuda.synchronize()
    plain.close()
    graph.close()


@pytest.mark.parametrize("prec", [hs.SPLIT_BF16, hs.SPLIT_INT8])
def test_lookahead_step_calls_use_set_of_the_panel(prec):
    # the step calls of a look-ahead plan keep panel g in set g % 2: outer
    # updates equal the plain plan's, and after a run the sets still hold
    # the last two panels, whose product launches alone reproduce the plain
    # plan's
    import torch
    n, P, Q, G, b, M = 512, 2, 2, 2, 32, 128
    _say("case lookahead step calls prec=%d" % prec)
    A = dev(inputs.uniform(n, n, 61))
    B = dev(inputs.uniform(n, n, 62))
    plain, ahead = _pair(n, P, Q, G, b, M, prec)
    wp, wa = plain.workspace(), ahead.workspace()
    Cp = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    Ca = torch.zeros_like(Cp)
    for g in range(plain.num_outer_steps):
        plain.outer_update(g, A, B, Cp, ws=wp)
        ahead.outer_update(g, A, B, Ca, ws=wa)
    torch.cuda.synchronize()
    assert torch.equal(Ca, Cp)
    _run(plain, A, B, ws=wp)
    _run(ahead, A, B, ws=wa)
    last = plain.num_outer_steps - 1
    for g in (last, last - 1):
        if g != last:
            # the plain plan's one set holds the last panel: split panel g again
            plain.outer_update(g, A, B, torch.zeros_like(Cp), ws=wp)
        Cp.zero_()
        Ca.zero_()
        plain.outer_products(g, A, B, Cp, wp)
        ahead.outer_products(g, A, B, Ca, wa)   # still in set g % 2 after the run
        torch.cuda.synchronize()
        assert torch.equal(Ca, Cp), g
    plain.close()
    ahead.close()


@pytest.mark.parametrize("n,k", [(1024, 4096), (4096, 2048)])
def test_lookahead_auto_equals_plain(n, k):
    # lookahead = 2 overlaps only where one product launch has fewer work
    # items than CUs (n = 1024: 128 items of 64 x 128; n = 4096: 2048); the
    # result is the plain one either way
    import torch
    P, Q, G, b, M = 4, 4, 4, 256, 1024
    _say("case lookahead auto n=%d k=%d" % (n, k))
    A = dev(inputs.exponent_spread(n, k, 81, 2.0))
    B = dev(inputs.exponent_spread(k, n, 82, 2.0))
    plain = hs.Plan(n, P, Q, G, b, M, k=k, prec=hs.SPLIT_INT8)
    auto = hs.Plan(n, P, Q, G, b, M, k=k, prec=hs.SPLIT_INT8, lookahead=2)
    ref, _ = _run(plain, A, B)
    got, _ = _run(auto, A, B)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    plain.close()
    auto.close()


def test_lookahead_noalloc():
    import torch
    n, P, Q, G, b, M = 640, 2, 2, 4, 32, 128
    _say("case lookahead noalloc n=%d INT8" % n)
    A = dev(inputs.exponent_spread(n, n, 71, 2.0))
    B = dev(inputs.exponent_spread(n, n, 72, 2.0))
    plain, ahead = _pair(n, P, Q, G, b, M, hs.SPLIT_INT8)
    ref, _ = _run(plain, A, B)
    C = torch.full_like(ref, float("nan"))
    ahead.run_noalloc(A, B, C)
    torch.cuda.synchronize()
    assert torch.equal(C, ref)
    plain.close()
    ahead.close()


@settings(max_examples=30, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(plans(), st.sampled_from([hs.SPLIT_BF16, hs.SPLIT_INT8]), st.integers(0, 2 ** 31 - 1))
def test_random_lookahead_equals_plain(c, prec, seed):
    import torch
    print("case random lookahead prec=%d %r" % (prec, c), flush=True)
    d = hs.DIST_BLOCK if c["dist"] == "block" else hs.DIST_BLOCK_CYCLIC
    kw = dict(m=c["m"], k=c["k"], dist=d, nb=c["nb"], persistent=c["persistent"])
    A = dev(inputs.exponent_spread(c["m"], c["k"], seed, 2.0))
    B = dev(inputs.exponent_spread(c["k"], c["n"], seed + 1, 2.0))
    plain, ahead = _pair(c["n"], c["P"], c["Q"], c["G"], c["b"], c["M"], prec, **kw)
    ref, _ = _run(plain, A, B)
    got, _ = _run(ahead, A, B)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    plain.close()
    ahead.close()
