"""GPU test of hsumma_run_noalloc, the entry point for callers that cannot
allocate: the product with the library's scratch array as workspace must
equal hsumma_run with a caller workspace, bit for bit, on two calls in a
row (the second smaller, so it must not depend on what the first left in
the shared array), for the FP64 path and the split forms."""
import sys

import numpy as np
import pytest

from paper_1306_4161_amd import hsumma as hs
from paper_1306_4161_amd import inputs

from gpu_helpers import dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [hs.FP64, hs.SPLIT_INT8, hs.SPLIT_BF16])
def test_noalloc_equals_run(prec):
    import torch
    limit = hs.lib().hsumma_noalloc_max_workspace()
    assert limit == 64 << 20
    for shape in ((1536, 3, 4, 6, 64, 256, 2.0), (640, 2, 2, 4, 32, 128, 0.0)):
        n, P, Q, G, b, M, sigma = shape
        print("case noalloc prec=%d %r" % (prec, shape), flush=True)
        sys.stdout.flush()
        if sigma:
            A = dev(inputs.exponent_spread(n, n, 161, sigma))
            B = dev(inputs.exponent_spread(n, n, 162, sigma))
        else:
            A = dev(inputs.uniform(n, n, 161))
            B = dev(inputs.uniform(n, n, 162))
        p = hs.Plan(n, P, Q, G, b, M, prec=prec)
        assert p.workspace_size <= limit
        ref = torch.empty((n, n), dtype=torch.float64, device="cuda")
        p.run(A, B, ref, ws=p.workspace())
        C = torch.full_like(ref, float("nan"))
        p.run_noalloc(A, B, C)
        torch.cuda.synchronize()
        assert torch.equal(C, ref)
        assert np.isfinite(C.cpu().numpy()).all()
        p.close()


def test_noalloc_equals_run_random_plans():
    # random plans (the strategy of tests/test_items_random.py), run back to
    # back through the one shared scratch array
    import torch
    from hypothesis import given, settings, strategies as st, HealthCheck
    from test_items_random import plans

    @settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])
    @given(plans(), st.integers(0, 2 ** 31 - 1))
    def check(c, seed):
        d = hs.DIST_BLOCK if c["dist"] == "block" else hs.DIST_BLOCK_CYCLIC
        p = hs.Plan(c["n"], c["P"], c["Q"], c["G"], c["b"], c["M"], m=c["m"], k=c["k"], dist=d,
                    nb=c["nb"], prec=c["prec"], persistent=c["persistent"])
        A = dev(inputs.uniform(c["m"], c["k"], seed))
        B = dev(inputs.uniform(c["k"], c["n"], seed + 1))
        ref = torch.empty((c["m"], c["n"]), dtype=torch.float64, device="cuda")
        p.run(A, B, ref, ws=p.workspace())
        C = torch.full_like(ref, float("nan"))
        p.run_noalloc(A, B, C)
        torch.cuda.synchronize()
        assert torch.equal(C, ref), c
        p.close()

    print("case noalloc random plans", flush=True)
    check()
