"""Randomized GPU parity (hypothesis): random shapes, grids, groupings,
distributions, macro-tiles and step sizes, every entry of C against the
oracle's Dot2.

  * FP64: within gamma_K (|A||B|)_ij (Sec. II-A's c_ij = sum_k a_ik b_kj;
    the classic bound of any FP64 dot product);
  * the BF16 and INT8 digit splits with automatic slice counts, on uniform
    and exponent-spread (sigma = 2) entries: max |c_hat - c| / (|A||B|)_ij
    <= 1e-14, the accuracy the slice-count policy is built for.
"""
import sys

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

from oracle import core
from paper_1306_4161_amd import hsumma as hs
from paper_1306_4161_amd import inputs

from gpu_helpers import check_sampled, dev, host
from test_items_random import plans

pytestmark = pytest.mark.gpu

GATE = 1e-14
TILES = [(0, 0, 0), (128, 128, 16), (128, 64, 16), (64, 128, 16), (64, 64, 16), (64, 64, 32),
         (32, 32, 16), (128, 128, 8), (256, 128, 16), (128, 256, 16)]


def _run(c, prec, A, B, tile=(0, 0, 0)):
    import torch
    d = hs.DIST_BLOCK if c["dist"] == "block" else hs.DIST_BLOCK_CYCLIC
    tm, tn, kc = tile
    p = hs.Plan(c["n"], c["P"], c["Q"], c["G"], c["b"], c["M"], m=c["m"], k=c["k"], dist=d,
                nb=c["nb"], prec=prec, persistent=c["persistent"], tile_m=tm, tile_n=tn, kc=kc)
    C = torch.empty((c["m"], c["n"]), dtype=torch.float64, device="cuda")
    C.fill_(float("nan"))
    p.run(dev(A), dev(B), C, ws=p.workspace())
    out = host(C)
    p.close()
    return out


@settings(max_examples=100, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(plans(), st.sampled_from(TILES), st.integers(0, 2 ** 31 - 1))
def test_random_fp64_within_bound(c, tile, seed):
    print("case random fp64 %r tile %r" % (c, tile), flush=True)
    A = inputs.uniform(c["m"], c["k"], seed)
    B = inputs.uniform(c["k"], c["n"], seed + 1)
    Ch = _run(c, hs.FP64, A, B, tile)
    rows, cols = np.meshgrid(np.arange(c["m"]), np.arange(c["n"]), indexing="ij")
    check_sampled(A, B, Ch, rows.ravel(), cols.ravel())


@settings(max_examples=100, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(plans(), st.sampled_from([hs.SPLIT_BF16, hs.SPLIT_INT8]), st.sampled_from([0.0, 2.0]),
       st.integers(0, 2 ** 31 - 1))
def test_random_splits_meet_gate(c, prec, sigma, seed):
    print("case random split prec=%d sigma=%g %r" % (prec, sigma, c), flush=True)
    if sigma > 0:
        A = inputs.exponent_spread(c["m"], c["k"], seed, sigma)
        B = inputs.exponent_spread(c["k"], c["n"], seed + 1, sigma)
    else:
        A = inputs.uniform(c["m"], c["k"], seed)
        B = inputs.uniform(c["k"], c["n"], seed + 1)
    Ch = _run(c, prec, A, B)
    rows, cols = np.meshgrid(np.arange(c["m"]), np.arange(c["n"]), indexing="ij")
    rows, cols = rows.ravel(), cols.ravel()
    ref, s = core.sampled(A, B, rows, cols)
    got = Ch[rows, cols]
    assert np.all(np.isfinite(got))
    with np.errstate(divide="ignore", invalid="ignore"):
        sc = np.where(s > 0, np.abs(got - ref) / s, np.abs(got - ref))
    assert float(sc.max()) <= GATE, "max scaled err %g" % float(sc.max())


@settings(max_examples=30, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(plans(), st.integers(0, 2 ** 31 - 1))
def test_random_graph_replays_equal_direct_launches(c, seed):
    # hsumma_run captured in a HIP graph (the work-item table regenerated on
    # every replay) against the direct launches, bit for bit, with eager work
    # and a dirtied workspace between replays
    import torch
    print("case random graph %r" % (c,), flush=True)
    d = hs.DIST_BLOCK if c["dist"] == "block" else hs.DIST_BLOCK_CYCLIC
    kw = dict(m=c["m"], k=c["k"], dist=d, nb=c["nb"], prec=c["prec"],
              persistent=c["persistent"])
    A = dev(inputs.uniform(c["m"], c["k"], seed))
    B = dev(inputs.uniform(c["k"], c["n"], seed + 1))
    direct = hs.Plan(c["n"], c["P"], c["Q"], c["G"], c["b"], c["M"], **kw)
    ref = torch.empty((c["m"], c["n"]), dtype=torch.float64, device="cuda")
    ws_direct = direct.workspace()
    direct.run(A, B, ref, ws=ws_direct)
    graph = hs.Plan(c["n"], c["P"], c["Q"], c["G"], c["b"], c["M"], use_graph=1, **kw)
    ws = graph.workspace()
    stream = torch.cuda.Stream()
    C = torch.empty_like(ref)
    for rep in range(3):
        # the side stream starts after everything queued on the default
        # stream (the direct run, the eager add): memory the caching
        # allocator hands out there may still be in use by that work
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            C.fill_(float("nan"))
            ws.fill_(0x5A + rep)
            graph.run(A, B, C, ws=ws, stream=stream)
        stream.synchronize()
        assert torch.equal(C, ref)
        A.add_(0.0)
    torch.cuda.synchronize()
    direct.close()
    graph.close()
