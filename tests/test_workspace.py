"""GPU checks of the workspace contract: the library allocates no device
memory; every compute call writes the plan's work-item table into the
caller's workspace with a kernel, then runs the update on it.

  * the table the device writes equals the plan's host definition bit for
    bit (group order, macro-tile blocks, XCD lists, longest-first order);
  * results do not depend on what the workspace held before a call (a
    workspace filled with garbage, or shared by two plans in turn, gives the
    same bits as a fresh one).
"""
import sys

import numpy as np
import pytest

from paper_1306_4161_amd import hsumma as hs
from paper_1306_4161_amd import inputs

from gpu_helpers import dev, host
from test_abi import ITEM_CASES

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


BIG = [
    (16384, 16, 16, 16, 256, 1024, "block", 0, 0, 0, {}),
    (16384, 16, 16, 16, 256, 1024, "block", 0, 0, 0, {"prec": hs.SPLIT_INT8}),
    (10000, 6, 10, 1, 128, 128, "cyclic", 128, 0, 0, {"prec": hs.SPLIT_BF16}),
]


@pytest.mark.parametrize("case", ITEM_CASES + BIG)
def test_device_table_equals_host_definition(case):
    import torch
    n, P, Q, G, b, M, dist, nb, m, k, extra = case
    _say("case table %r" % (case,))
    d = hs.DIST_BLOCK if dist == "block" else hs.DIST_BLOCK_CYCLIC
    p = hs.Plan(n, P, Q, G, b, M, dist=d, nb=nb, m=m, k=k, **extra)
    ws = p.workspace()
    ws.fill_(0xA5)
    p.prepare_workspace(ws)
    torch.cuda.synchronize()
    nit = p.num_items
    got = ws[:16 * nit].view(torch.int32).cpu().numpy().reshape(nit, 4)
    assert np.array_equal(got, p.work_items())
    p.close()


@pytest.mark.parametrize("prec", [hs.FP64, hs.SPLIT_INT8, hs.SPLIT_BF16])
def test_results_independent_of_workspace_contents(prec):
    import torch
    _say("case dirty workspace prec=%d" % prec)
    n = 640
    A, B = dev(inputs.uniform(n, n, 61)), dev(inputs.uniform(n, n, 62))
    p = hs.Plan(n, 2, 5, 10, 32, 128, prec=prec)
    q = hs.Plan(n, 5, 2, 1, 64, 64, prec=prec, persistent=1)
    ref_p = torch.empty((n, n), dtype=torch.float64, device="cuda")
    ref_q = torch.empty_like(ref_p)
    p.run(A, B, ref_p, ws=p.workspace())
    q.run(A, B, ref_q, ws=q.workspace())
    # one workspace, large enough for both plans, shared in turn and dirtied
    shared = torch.empty(max(p.workspace_size, q.workspace_size) + 4096, dtype=torch.uint8,
                         device="cuda")
    C = torch.empty_like(ref_p)
    for rep in range(2):
        shared.fill_(0x5A + rep)
        p.run(A, B, C, ws=shared)
        assert torch.equal(C, ref_p)
        q.run(A, B, C, ws=shared)
        assert torch.equal(C, ref_q)
    # the step calls regenerate the table too
    C.zero_()
    for s in range(p.num_steps):
        shared.fill_(0x33)
        p.local_update(s, A, B, C, ws=shared)
    C2 = torch.zeros_like(C)
    wsp = p.workspace()
    for s in range(p.num_steps):
        p.local_update(s, A, B, C2, ws=wsp)
    assert torch.equal(C, C2)
    assert np.isfinite(host(C)).all()


def test_device_table_equals_host_definition_random_plans():
    # random shapes, grids, groupings, distributions and precisions (the
    # strategy of tests/test_items_random.py), each table written by the
    # device generator into a dirtied workspace
    import torch
    from hypothesis import given, settings, HealthCheck
    from test_items_random import plans

    @settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
    @given(plans())
    def check(c):
        d = hs.DIST_BLOCK if c["dist"] == "block" else hs.DIST_BLOCK_CYCLIC
        p = hs.Plan(c["n"], c["P"], c["Q"], c["G"], c["b"], c["M"], m=c["m"], k=c["k"], dist=d,
                    nb=c["nb"], prec=c["prec"], persistent=c["persistent"])
        ws = p.workspace()
        ws.fill_(0x3C)
        p.prepare_workspace(ws)
        torch.cuda.synchronize()
        nit = p.num_items
        got = ws[:16 * nit].view(torch.int32).cpu().numpy().reshape(nit, 4)
        assert np.array_equal(got, p.work_items()), c
        p.close()

    _say("case random device tables")
    check()


def test_workspace_helpers_return_4k_aligned_buffers():
    # the bindings' workspace helpers honour the recommended 4 KiB alignment
    # (the caching allocator alone hands out blocks at 512-byte offsets)
    import torch
    keep = [torch.empty(1536 + 512 * i, dtype=torch.uint8, device="cuda") for i in range(4)]
    for prec in (hs.FP64, hs.SPLIT_INT8):
        p = hs.Plan(640, 2, 2, 4, 32, 128, prec=prec)
        for _ in range(3):
            ws = p.workspace()
            assert ws.data_ptr() % 4096 == 0 and ws.numel() == p.workspace_size
        p.close()
    lu = hs.LuPlan(512, 2, 2, 4, 32, 128)
    assert lu.workspace().data_ptr() % 4096 == 0
    lu.close()
    del keep
