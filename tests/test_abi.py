"""Host-side checks of the C ABI: exported symbols, validation, plan math.

No GPU needed: plan creation and queries are host-only.  The plan's step
schedule, owner map, grouping and tile shapes are compared with the oracle's
independent plan reference (oracle/plan_ref.py).
"""
import ctypes
import os
import re

import pytest

from oracle import plan_ref
from paper_1306_4161_amd import hsumma as hs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(hsumma_\w+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(hs.LIB_PATH)
    declared = _declared_functions()
    assert "hsumma_plan" in declared and "hsumma_local_update" in declared
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(hs.EXPORTED) <= declared | {"hsumma_opts_default"}


def test_version():
    assert hs.version().startswith("hsumma-gfx950")


@pytest.mark.parametrize("args,msg", [
    ((100, 4, 4, 3, 8, 8), "cannot be arranged"),
    ((100, 4, 4, 1, 0, 8), "b must be"),
    ((100, 4, 4, 1, 16, 8), "M must be >="),
    ((100, 4, 4, 1, 16, 24), "multiple of b"),
    ((3, 4, 1, 1, 1, 1), "grid larger"),
    ((0, 1, 1, 1, 1, 1), "positive"),
    ((64, 2, 3, 4, 8, 8), "cannot be arranged"),
])
def test_plan_rejects_invalid(args, msg):
    with pytest.raises(hs.HsummaError) as ei:
        hs.Plan(*args)
    assert ei.value.code == hs.ERR_INVALID
    assert msg in str(ei.value)


def test_plan_rejects_sizes_beyond_32_bits():
    for kw in (dict(k=2 ** 31), dict(m=2 ** 31)):
        with pytest.raises(hs.HsummaError) as ei:
            hs.Plan(64, 1, 1, 1, 8, 8, **kw)
        assert ei.value.code == hs.ERR_INVALID
        assert "below 2^31" in str(ei.value)


def test_plan_rejects_unknown_tile_and_enum():
    with pytest.raises(hs.HsummaError):
        hs.Plan(256, 2, 2, 1, 32, tile_m=96, tile_n=96)
    with pytest.raises(hs.HsummaError):
        hs.Plan(256, 2, 2, 1, 32, dist=7)
    with pytest.raises(hs.HsummaError):
        hs.Plan(256, 2, 2, 1, 32, prec=9)
    with pytest.raises(hs.HsummaError) as ei:
        hs.Plan(256, 2, 2, 1, 32, wgs_per_cu=-1)
    assert "wgs_per_cu" in str(ei.value)


PLAN_CASES = [
    # n, P, Q, G, b, M, dist, nb, m, k
    (256, 2, 2, 1, 32, 32, "block", 0, 0, 0),
    (8192, 8, 8, 4, 64, 256, "block", 0, 0, 0),
    (16384, 16, 16, 16, 256, 256, "block", 0, 0, 0),
    (10000, 6, 10, 1, 128, 128, "cyclic", 128, 0, 0),
    (1000, 6, 6, 9, 20, 40, "block", 0, 0, 0),
    (77, 3, 5, 15, 6, 12, "cyclic", 5, 91, 53),
    (130, 4, 3, 6, 7, 21, "block", 0, 65, 200),
]


@pytest.mark.parametrize("case", PLAN_CASES)
def test_plan_matches_reference(case):
    n, P, Q, G, b, M, dist, nb, m, k = case
    d = hs.DIST_BLOCK if dist == "block" else hs.DIST_BLOCK_CYCLIC
    p = hs.Plan(n, P, Q, G, b, M, dist=d, nb=nb, m=m, k=k)
    m = m or n
    k = k or n
    nbe = nb or b
    assert p.groups == plan_ref.factor_groups(P, Q, G)
    ref_steps = plan_ref.steps(k, b, M)
    assert p.num_steps == len(ref_steps)
    assert p.num_outer_steps == len({s.outer for s in ref_steps})
    I, J = p.groups
    gp, gq = P // I, Q // J
    for s in ref_steps[:: max(1, len(ref_steps) // 50)] + ref_steps[-2:]:
        info = p.step_info(s.index)
        assert (info["k0"], info["k1"], info["outer"]) == (s.k0, s.k1, s.outer)
        q = plan_ref.owner(s.k0, k, Q, dist, nbe)
        r = plan_ref.owner(s.k0, k, P, dist, nbe)
        assert info["owner_col"] == q and info["owner_row"] == r
        assert (info["group_col"], info["in_group_col"]) == (q // gq, q % gq)
        assert (info["group_row"], info["in_group_row"]) == (r // gp, r % gp)
    if m * n <= 10 ** 8:
        shapes = plan_ref.tile_shapes(m, n, P, Q, dist, nbe) if m * n < 4 * 10 ** 6 else None
        for pr in range(P):
            for pc in range(Q):
                got = p.tile_shape(pr, pc)
                if shapes is not None:
                    assert got == shapes[(pr, pc)]
                else:
                    assert got == (len(plan_ref.local_indices(m, P, pr, dist, nbe)),
                                   len(plan_ref.local_indices(n, Q, pc, dist, nbe)))
    p.close()


def test_cyclic_tiles_of_the_6x10_grid():
    p = hs.Plan(10000, 6, 10, 1, 128, dist=hs.DIST_BLOCK_CYCLIC)
    rows = {p.tile_shape(r, 0)[0] for r in range(6)}
    cols = {p.tile_shape(0, c)[1] for c in range(10)}
    assert rows == {1680, 1664} and cols == {1024, 912, 896}
    assert p.num_steps == 79
    assert p.step_info(78)["k1"] - p.step_info(78)["k0"] == 16


def test_queries_reject_bad_indices():
    p = hs.Plan(64, 2, 2, 1, 8)
    with pytest.raises(hs.HsummaError):
        p.step_info(8)
    with pytest.raises(hs.HsummaError):
        p.tile_shape(2, 0)
    # every precision needs a workspace: at least the work-item table
    assert p.workspace_size >= 16 * p.num_items > 0


ITEM_CASES = [
    # n, P, Q, G, b, M, dist, nb, m, k, extra plan options
    (384, 3, 3, 3, 16, 64, "block", 0, 0, 0, {}),
    (1000, 6, 6, 9, 20, 40, "block", 0, 0, 0, {}),
    (1000, 6, 6, 9, 20, 40, "block", 0, 0, 0, {"persistent": 1}),
    (10000, 6, 10, 1, 128, 128, "cyclic", 128, 0, 0, {"persistent": 1}),
    (77, 3, 5, 15, 6, 12, "cyclic", 5, 91, 53, {}),
    (130, 4, 3, 6, 7, 21, "block", 0, 65, 200, {"persistent": 1}),
    (768, 3, 4, 6, 32, 128, "block", 0, 0, 0, {"prec": hs.SPLIT_INT8}),
    (700, 2, 3, 2, 50, 100, "cyclic", 70, 500, 0, {"prec": hs.SPLIT_BF16}),
    (512, 4, 4, 16, 32, 64, "block", 0, 0, 0, {"tile_m": 32, "tile_n": 32}),
]


@pytest.mark.parametrize("case", ITEM_CASES)
def test_work_items_cover_c_once_inside_one_tile(case):
    # The work-item table (Sec. II-A: each processor updates its own block of
    # C; Sec. III: processors listed group by group): the macro-tiles cover
    # every entry of C exactly once, each lies in one processor's tile and in
    # one distribution block, and in the longest-first modes every XCD list
    # has non-increasing areas.
    import numpy as np
    n, P, Q, G, b, M, dist, nb, m, k, extra = case
    d = hs.DIST_BLOCK if dist == "block" else hs.DIST_BLOCK_CYCLIC
    p = hs.Plan(n, P, Q, G, b, M, dist=d, nb=nb, m=m, k=k, **extra)
    m = m or n
    nbe = nb or b
    it = p.work_items()
    assert it.shape == (p.num_items, 4)
    assert p.workspace_size >= 16 * p.num_items
    cover = np.zeros((m, n), dtype=np.int32)
    for r0, c0, h, w in it:
        assert h > 0 and w > 0
        cover[r0:r0 + h, c0:c0 + w] += 1
        pr = plan_ref.owner(r0, m, P, dist, nbe)
        pc = plan_ref.owner(c0, n, Q, dist, nbe)
        assert plan_ref.owner(r0 + h - 1, m, P, dist, nbe) == pr
        assert plan_ref.owner(c0 + w - 1, n, Q, dist, nbe) == pc
        if dist == "cyclic":
            assert r0 // nbe == (r0 + h - 1) // nbe and c0 // nbe == (c0 + w - 1) // nbe
    assert cover.min() == 1 and cover.max() == 1
    per = (p.num_items + 7) // 8
    if extra.get("persistent") or extra.get("prec"):
        for x in range(8):
            a = it[x * per:(x + 1) * per, 2].astype(np.int64) * it[x * per:(x + 1) * per, 3]
            assert np.all(a[:-1] >= a[1:])
    p.close()


def test_compute_calls_check_the_workspace_before_launching():
    # host-side validation: a missing, short or misaligned workspace is
    # rejected before anything is launched (fake device addresses suffice)
    import ctypes
    p = hs.Plan(256, 2, 2, 1, 32)
    L = hs.lib()
    A, B, C = (ctypes.c_void_p(0x100000 * (i + 1)) for i in range(3))
    need = p.workspace_size
    cases = [(None, need, hs.ERR_WORKSPACE), (0x7000000, need - 1, hs.ERR_WORKSPACE),
             (0x7000010, need, hs.ERR_INVALID)]
    for wsp, wsn, code in cases:
        ws = ctypes.c_void_p(wsp)
        assert L.hsumma_run(p._h, A, 256, B, 256, C, 256, ws, wsn, None) == code
        assert L.hsumma_local_update(p._h, 0, A, 256, B, 256, C, 256, ws, wsn, None) == code
        assert L.hsumma_outer_update(p._h, 0, A, 256, B, 256, C, 256, ws, wsn, None) == code
        assert L.hsumma_prepare_workspace(p._h, ws, wsn, None) == code
    p.close()


def test_split_plans_validate_slices_panel_and_steps():
    # host-only: plan validation and workspace sizing of the three digit formats
    n, M = 512, 256
    for prec, smax, esz in ((hs.SPLIT_BF16, 7, 2), (hs.SPLIT_FP8, 7, 1), (hs.SPLIT_INT8, 8, 1)):
        p = hs.Plan(n, 2, 2, 1, 64, M, prec=prec)
        lay = p.split_layout()
        assert lay["planes"] == smax and lay["Wp"] % 32 == 0
        # the digit planes of both operands fit in the workspace
        assert p.workspace_size >= 2 * smax * n * lay["Wp"] * esz
        p.close()
        hs.Plan(n, 2, 2, 1, 64, M, prec=prec, slices=smax, min_slices=1).close()
        with pytest.raises(hs.HsummaError) as ei:
            hs.Plan(n, 2, 2, 1, 64, M, prec=prec, max_slices=smax + 1)
        assert ei.value.code == hs.ERR_INVALID
        with pytest.raises(hs.HsummaError):
            hs.Plan(n, 2, 2, 1, 64, M, prec=prec, slices=smax + 1)
    # exact accumulation over a panel bounds M for the FP8 and INT8 forms
    for prec in (hs.SPLIT_FP8, hs.SPLIT_INT8):
        hs.Plan(16384, 2, 2, 1, 64, 8192, prec=prec).close()
        with pytest.raises(hs.HsummaError) as ei:
            hs.Plan(16384, 2, 2, 1, 64, 16384, prec=prec)
        assert "M <= 8192" in str(ei.value)
    hs.Plan(16384, 2, 2, 1, 64, 16384, prec=hs.SPLIT_BF16).close()
    # the INT8 form streams 32-k steps, the others 16-k steps
    hs.Plan(n, 2, 2, 1, 64, M, prec=hs.SPLIT_INT8, kc=32).close()
    hs.Plan(n, 2, 2, 1, 64, M, prec=hs.SPLIT_BF16, kc=16).close()
    for prec, kc in ((hs.SPLIT_INT8, 16), (hs.SPLIT_BF16, 32)):
        with pytest.raises(hs.HsummaError):
            hs.Plan(n, 2, 2, 1, 64, M, prec=prec, kc=kc)


def test_noalloc_rejects_a_plan_beyond_its_scratch_array():
    # host-side: the check precedes any device call (fake device addresses)
    import ctypes
    L = hs.lib()
    limit = L.hsumma_noalloc_max_workspace()
    assert limit == 64 << 20
    big = hs.Plan(16384, 16, 16, 16, 256, 1024, prec=hs.SPLIT_INT8)
    assert big.workspace_size > limit
    A, B, C = (ctypes.c_void_p(0x100000 * (i + 1)) for i in range(3))
    assert L.hsumma_run_noalloc(big._h, A, 16384, B, 16384, C, 16384, None) == hs.ERR_WORKSPACE
    assert "scratch" in L.hsumma_last_error().decode()
    big.close()


def test_digit_planes_start_on_4k_boundaries():
    # the plane sets (and their partial statistics) sit on 4 KiB boundaries of
    # the workspace, whatever the item table before them
    for n, P, Q, G, b, M, prec in [(700, 3, 2, 2, 32, 96, hs.SPLIT_INT8),
                                   (1000, 4, 4, 4, 64, 256, hs.SPLIT_BF16),
                                   (333, 1, 3, 3, 16, 48, hs.SPLIT_FP8)]:
        p = hs.Plan(n, P, Q, G, b, M, prec=prec)
        lay = p.split_layout()
        assert lay["off_digA"] % 4096 == 0 and lay["off_digB"] % 4096 == 0
        p.close()


def test_split_outer_block_fits_the_split_grid():
    # one grid row of the split kernels per 64 panel columns, at most 65535
    hs.Plan(64, 1, 1, 1, 64, 65535 * 64, k=65535 * 64, prec=hs.SPLIT_BF16).close()
    with pytest.raises(hs.HsummaError):
        hs.Plan(64, 1, 1, 1, 64, 65535 * 64 + 64, k=65535 * 64 + 64, prec=hs.SPLIT_BF16)


def test_split_lookahead_doubles_the_panel_sets():
    # look-ahead in a split form: a second set of digit planes (max_slices
    # planes of m x Wp and n x Wp digits), exponents and partial statistics;
    # nothing for FP64
    al = lambda x: (x + 255) // 256 * 256
    for prec, esz, planes in ((hs.SPLIT_BF16, 2, 7), (hs.SPLIT_INT8, 1, 8)):
        m, n, k, M = 600, 520, 1000, 128
        plain = hs.Plan(n, 2, 2, 4, 32, M, m=m, k=k, prec=prec)
        ahead = hs.Plan(n, 2, 2, 4, 32, M, m=m, k=k, prec=prec, lookahead=1)
        Wp = 128
        part = 6 * (Wp // 64) * (m + n) * 8       # per-slab partial statistics
        extra = (al(planes * m * Wp * esz) + al(planes * n * Wp * esz) + al(4 * m) + al(4 * n)
                 + al(part))
        # (up to three 4 KiB roundings: each plane set and the partial
        # statistics start on a 4 KiB boundary)
        assert 0 <= ahead.workspace_size - plain.workspace_size - extra <= 3 * 4096
        assert ahead.work_items().tolist() == plain.work_items().tolist()
        plain.close(); ahead.close()
    f0 = hs.Plan(512, 2, 2, 4, 32, 128)
    f1 = hs.Plan(512, 2, 2, 4, 32, 128, lookahead=1)
    assert f1.workspace_size == f0.workspace_size
    f0.close(); f1.close()
    # 2: the automatic mode (decided per call) needs the same workspace as 1
    a1 = hs.Plan(512, 2, 2, 4, 32, 128, prec=hs.SPLIT_INT8, lookahead=1)
    a2 = hs.Plan(512, 2, 2, 4, 32, 128, prec=hs.SPLIT_INT8, lookahead=2)
    assert a2.workspace_size == a1.workspace_size
    a1.close(); a2.close()
    for bad in (-1, 3):
        with pytest.raises(hs.HsummaError):
            hs.Plan(512, 2, 2, 4, 32, 128, prec=hs.SPLIT_INT8, lookahead=bad)


def test_lu_plans_validate_and_size_their_workspace():
    with pytest.raises(hs.HsummaError):
        hs.LuPlan(256, 1, 1, 1, 128, 128)            # b beyond the 64 of the panel kernels
    with pytest.raises(hs.HsummaError):
        hs.LuPlan(256, 1, 1, 1, 32, 48)              # M not a multiple of b
    with pytest.raises(hs.HsummaError):
        hs.LuPlan(256, 1, 1, 1, 32, 16)              # M < b
    p = hs.LuPlan(1000, 4, 4, 16, 64, 256)
    # the negated L21 panel (n x M doubles) plus the trailing updates' workspace
    assert p.workspace_size >= 1000 * 256 * 8 + 16 * ((1000 - 256 + 127) // 128) ** 2
    q = hs.LuPlan(1000, 4, 4, 16, 64, 256, prec=hs.SPLIT_INT8)
    assert q.workspace_size > p.workspace_size       # digit planes of the trailing updates
    # look-ahead: two L21 buffers and a second region for the concurrent update
    la = hs.LuPlan(1000, 4, 4, 16, 64, 256, lookahead=1)
    assert la.workspace_size >= 2 * 1000 * 256 * 8 + 2 * 256
    assert la.workspace_size > p.workspace_size
    la.close()
    one = hs.LuPlan(200, 4, 4, 16, 64, 256, lookahead=1)   # one panel: nothing to overlap
    assert one.workspace_size >= 2 * 200 * 256 * 8
    one.close()
    import ctypes
    ws = ctypes.c_void_p(0x7000000)
    A = ctypes.c_void_p(0x100000)
    assert hs.lib().hsumma_lu(p._h, A, 1000, ws, p.workspace_size - 1, None) == hs.ERR_WORKSPACE
    assert hs.lib().hsumma_lu(p._h, A, 999, ws, p.workspace_size, None) == hs.ERR_INVALID
    p.close(); q.close()


def test_plans_accept_the_compiled_tiles_and_wave_counts():
    for tm, tn, kc, w in [(128, 256, 16, 0), (64, 256, 16, 0), (256, 64, 16, 0),
                          (128, 128, 16, 8), (128, 128, 16, 4)]:
        hs.Plan(1024, 2, 2, 4, 64, 128, tile_m=tm, tile_n=tn, kc=kc, waves=w).close()
    for tm, tn, kc, w in [(256, 256, 16, 0), (128, 128, 16, 2), (128, 128, 16, 16)]:
        with pytest.raises(hs.HsummaError):
            hs.Plan(1024, 2, 2, 4, 64, 128, tile_m=tm, tile_n=tn, kc=kc, waves=w)


@pytest.mark.parametrize("args,kw,tile", [
    ((16384, 16, 16, 16, 256, 1024), {}, (128, 64, 16)),      # outer block >= 1024
    ((16384, 16, 16, 16, 256, 256), {}, (128, 128, 16)),
    ((8192, 8, 8, 4, 64, 256), {}, (128, 128, 16)),
    ((10000, 6, 10, 1, 128, 128), {"dist": hs.DIST_BLOCK_CYCLIC}, (128, 128, 16)),
    ((6000, 16, 16, 16, 512, 512), {}, (64, 64, 16)),        # processor tiles of 375
    ((16384, 16, 16, 16, 64, 64), {}, (64, 64, 16)),         # outer block under 128
    ((256, 2, 2, 1, 32, 32), {}, (32, 32, 16)),              # 16 items of 64 x 64
    ((16384, 16, 16, 16, 256, 1024), {"kc": 32}, (128, 128, 32)),
    ((16384, 16, 16, 16, 256, 1024), {"tile_m": 256, "tile_n": 128, "kc": 8}, (256, 128, 8)),
    ((16384, 16, 16, 16, 256, 1024), {"prec": hs.SPLIT_INT8}, (64, 128, 32)),
    ((16384, 16, 16, 16, 256, 1024), {"prec": hs.SPLIT_BF16}, (64, 128, 16)),
])
def test_default_tile_rule(args, kw, tile):
    # the macro-tile the plan picks when none is named (hsumma_tile_config)
    p = hs.Plan(*args, **kw)
    tm, tn, kc, waves = p.tile_config
    assert (tm, tn, kc) == tile and waves > 0
    p.close()
