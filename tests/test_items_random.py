"""Randomized checks of the work-item table on the CPU (the plan's host
definition, hsumma_work_items; the device generator is compared with it bit
for bit by tests/test_workspace.py).

For random shapes, grids, groupings, distributions, precisions and the
default macro-tile rule: the macro-tiles cover every entry of C exactly once
(Sec. II-A: every processor updates its own block), each lies in one
processor's tile and one distribution block, the table lists processors
group by group (Sec. III) unless the longest-first order applies, and in
that order every XCD list has non-increasing areas.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

from oracle import plan_ref
from paper_1306_4161_amd import hsumma as hs


def _groups(P, Q):
    return sorted({I * J for I in range(1, P + 1) if P % I == 0
                   for J in range(1, Q + 1) if Q % J == 0})


@st.composite
def plans(draw):
    P = draw(st.integers(1, 6))
    Q = draw(st.integers(1, 6))
    m = draw(st.integers(P, 400))
    n = draw(st.integers(Q, 400))
    k = draw(st.integers(1, 300))
    G = draw(st.sampled_from(_groups(P, Q)))
    b = draw(st.integers(1, 64))
    M = b * draw(st.integers(1, 4))
    dist = draw(st.sampled_from(["block", "cyclic"]))
    nb = draw(st.integers(1, 96)) if dist == "cyclic" else 0
    prec = draw(st.sampled_from([hs.FP64, hs.FP64, hs.SPLIT_INT8, hs.SPLIT_BF16]))
    persistent = draw(st.integers(0, 1))
    return dict(n=n, P=P, Q=Q, G=G, b=b, M=M, m=m, k=k, dist=dist, nb=nb, prec=prec,
                persistent=persistent)


@settings(max_examples=120, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(plans())
def test_random_tables_cover_c_once_in_group_order(c):
    d = hs.DIST_BLOCK if c["dist"] == "block" else hs.DIST_BLOCK_CYCLIC
    p = hs.Plan(c["n"], c["P"], c["Q"], c["G"], c["b"], c["M"], m=c["m"], k=c["k"], dist=d,
                nb=c["nb"], prec=c["prec"], persistent=c["persistent"])
    m, n, P, Q = c["m"], c["n"], c["P"], c["Q"]
    nbe = c["nb"] or c["b"]
    I, J = plan_ref.factor_groups(P, Q, c["G"])
    assert p.groups == (I, J)
    tm, tn, _, _ = p.tile_config
    it = p.work_items()
    assert it.shape == (p.num_items, 4)
    cover = np.zeros((m, n), dtype=np.int32)
    ranks = []
    for r0, c0, h, w in it:
        assert 0 < h <= tm and 0 < w <= tn
        cover[r0:r0 + h, c0:c0 + w] += 1
        pr = plan_ref.owner(r0, m, P, c["dist"], nbe)
        pc = plan_ref.owner(c0, n, Q, c["dist"], nbe)
        assert plan_ref.owner(r0 + h - 1, m, P, c["dist"], nbe) == pr
        assert plan_ref.owner(c0 + w - 1, n, Q, c["dist"], nbe) == pc
        if c["dist"] == "cyclic":
            assert r0 // nbe == (r0 + h - 1) // nbe and c0 // nbe == (c0 + w - 1) // nbe
        x, y, i, j = plan_ref.group_coords(pr, pc, P, Q, I, J)
        ranks.append(((x * J + y) * (P // I) + i) * (Q // J) + j)
    assert cover.min() == 1 and cover.max() == 1
    per = (p.num_items + 7) // 8
    if c["persistent"] or c["prec"] != hs.FP64:
        for x in range(8):
            a = it[x * per:(x + 1) * per, 2].astype(np.int64) * it[x * per:(x + 1) * per, 3]
            assert np.all(a[:-1] >= a[1:])
    else:
        # group by group, processor by processor
        assert all(a <= b for a, b in zip(ranks, ranks[1:]))
    p.close()
