"""Pins of the communication-cost oracle (oracle/cost_model.py) to what the
paper and the mathematics fix.

The paper prints the same costs in several independent forms: the per-item
formulas of Sec. IV-A/IV-B, Tables I-II, the general model of eq. (2)-(5),
the derivative of eq. (10), the optimum of eq. (12) and the curves of
Fig. 10.  Each test ties two of those forms together, or one of them to a
statement of the paper (SUMMA is HSUMMA with G = 1 or G = p; the extremum at
G = sqrt(p) is a minimum iff alpha/beta > 2 n b / p), so that a dropped term,
a wrong sign or a wrong coefficient in any one of them fails.
"""
import math

import pytest

from oracle import cost_model as cm

# The paper's three platform parameter sets (Sec. V-A2, V-B1, V-C), with the
# readings of its garbles: Grid5000 p = 128 (the value its own check uses);
# "Bandwidth: 1E-9" on BG/P is the reciprocal bandwidth; exascale
# beta = 1 / (100 GB/s) per element as Fig. 10 applies it.
PLATFORMS = {
    "grid5000": dict(n=8192, p=128, b=64, alpha=1e-4, beta=1e-9),
    "bgp": dict(n=65536, p=16384, b=256, alpha=3e-6, beta=1e-9),
    "exascale": dict(n=2 ** 22, p=2 ** 20, b=256, alpha=5e-7, beta=1e-11),
}


def close(a, b, rel=1e-12):
    return abs(a - b) <= rel * max(abs(a), abs(b), 1e-300)


@pytest.mark.parametrize("name", sorted(PLATFORMS))
def test_summa_is_hsumma_with_one_or_p_groups(name):
    # Sec. IV-C: T_S is the special case G = 1 or G = p of T_HS (b = B)
    pf = PLATFORMS[name]
    n, p, b, al, be = pf["n"], pf["p"], pf["b"], pf["alpha"], pf["beta"]
    for hs, su in ((cm.hsumma_vdg, cm.summa_vdg), (cm.hsumma_binomial, cm.summa_binomial)):
        ref = sum(su(n, p, b, al, be))
        for G in (1, p):
            assert close(sum(hs(n, p, G, b, b, al, be)), ref)
    for L, W in ((cm.L_vdg, cm.W_vdg), (cm.L_binomial, cm.W_binomial)):
        ref = cm.T_S(n, p, b, L, W, al, be)
        for G in (1, p):
            assert close(cm.T_HS(n, p, G, b, L, W, al, be), ref)


@pytest.mark.parametrize("name", sorted(PLATFORMS))
def test_general_model_reproduces_the_tables(name):
    # eq. (2)-(5) with the binomial / Van de Geijn L, W against Sec. IV-A/B
    pf = PLATFORMS[name]
    n, p, b, al, be = pf["n"], pf["p"], pf["b"], pf["alpha"], pf["beta"]
    assert close(cm.T_S(n, p, b, cm.L_vdg, cm.W_vdg, al, be), sum(cm.summa_vdg(n, p, b, al, be)))
    assert close(cm.T_S(n, p, b, cm.L_binomial, cm.W_binomial, al, be),
                 sum(cm.summa_binomial(n, p, b, al, be)))
    for G in (2, 4, 16, 64, p // 4):
        assert close(cm.T_HS(n, p, G, b, cm.L_vdg, cm.W_vdg, al, be),
                     sum(cm.hsumma_vdg(n, p, G, b, b, al, be)))
        assert close(cm.T_HS(n, p, G, b, cm.L_binomial, cm.W_binomial, al, be),
                     sum(cm.hsumma_binomial(n, p, G, b, b, al, be)))


def test_broadcast_forms_agree_with_eq1():
    for p in (2, 3, 16, 1000):
        for m in (1.0, 64.0, 1e6):
            assert close(cm.bcast_binomial(m, p, 2e-6, 3e-9),
                         cm.L_binomial(p) * 2e-6 + m * cm.W_binomial(p) * 3e-9)
            assert close(cm.bcast_vdg(m, p, 2e-6, 3e-9),
                         cm.L_vdg(p) * 2e-6 + m * cm.W_vdg(p) * 3e-9)
    # a broadcast among one process costs nothing (L(1) = W(1) = 0, eq. (1))
    assert cm.bcast_binomial(5.0, 1, 1.0, 1.0) == 0.0 and cm.bcast_vdg(5.0, 1, 1.0, 1.0) == 0.0


@pytest.mark.parametrize("name", sorted(PLATFORMS))
def test_eq10_is_the_derivative_of_table2(name):
    pf = PLATFORMS[name]
    n, p, b, al, be = pf["n"], pf["p"], pf["b"], pf["alpha"], pf["beta"]

    def T(G):
        return sum(cm.hsumma_vdg(n, p, G, b, b, al, be))
    for G in (2.0, 7.5, math.sqrt(p), p / 3.0):
        h = G * 1e-5
        num = (T(G + h) - T(G - h)) / (2 * h)
        ana = cm.dTHS_dG_vdg(n, p, G, b, al, be)
        assert abs(num - ana) <= 1e-5 * max(abs(ana), abs(T(G)) / G)
    assert cm.dTHS_dG_vdg(n, p, math.sqrt(p), b, al, be) == 0.0


@pytest.mark.parametrize("name", sorted(PLATFORMS))
def test_eq12_is_table2_at_sqrt_p(name):
    pf = PLATFORMS[name]
    n, p, b, al, be = pf["n"], pf["p"], pf["b"], pf["alpha"], pf["beta"]
    assert close(cm.optimal_vdg(n, p, b, al, be),
                 sum(cm.hsumma_vdg(n, p, math.sqrt(p), b, b, al, be)), rel=1e-11)


def test_eq11_regimes():
    # the paper's printed thresholds: 2*8192*64/128 = 8192 (Grid5000); the
    # condition holds for all three platforms (Sec. V-A2, V-B1, V-C)
    g = PLATFORMS["grid5000"]
    assert 2 * g["n"] * g["b"] / g["p"] == 8192
    for name, pf in PLATFORMS.items():
        n, p, b, al, be = pf["n"], pf["p"], pf["b"], pf["alpha"], pf["beta"]
        assert cm.minimum_at_sqrt_p(n, p, b, al, be), name
        t_opt = sum(cm.hsumma_vdg(n, p, math.sqrt(p), b, b, al, be))
        for G in (2, 4, p / 8, p / 2):
            assert t_opt < sum(cm.hsumma_vdg(n, p, G, b, b, al, be)), (name, G)
        assert t_opt < sum(cm.summa_vdg(n, p, b, al, be))
    # below the threshold sqrt(p) is the maximum and SUMMA (G = 1) the best
    n, p, b = 8192, 256, 64
    al, be = 1e-7, 1e-9                       # alpha/beta = 100 < 2nb/p = 4096
    assert not cm.minimum_at_sqrt_p(n, p, b, al, be)
    t_mid = sum(cm.hsumma_vdg(n, p, 16, b, b, al, be))
    for G in (1, 2, 64, 256):
        assert t_mid > sum(cm.hsumma_vdg(n, p, G, b, b, al, be))


def test_binomial_cost_does_not_depend_on_G_when_b_equals_B():
    # log2(p/G) + log2(G) = log2(p): both factors of Table I are constant in G
    n, p, b = 4096, 1024, 128
    ref = sum(cm.summa_binomial(n, p, b, 1e-5, 1e-9))
    for G in (2, 32, 512):
        assert close(sum(cm.hsumma_binomial(n, p, G, b, b, 1e-5, 1e-9)), ref)
    # a larger outer block only lowers the between-groups latency
    t_bB = sum(cm.hsumma_binomial(n, p, 32, b, 4 * b, 1e-5, 1e-9))
    assert t_bB < ref


@pytest.mark.parametrize("name", sorted(PLATFORMS))
def test_fig10_curves_match_table2(name):
    pf = PLATFORMS[name]
    n, p, b, al, be = pf["n"], pf["p"], pf["b"], pf["alpha"], pf["beta"]
    gamma = 1e-18
    comp = 2 * n ** 3 * gamma / p
    for G in (1, 4, math.sqrt(p), p):
        hs, su = cm.exascale_plot(n, p, G, b, al, be, gamma)
        assert close(hs - comp, sum(cm.hsumma_vdg(n, p, G, b, b, al, be)), rel=1e-10)
        assert close(su - comp, sum(cm.summa_vdg(n, p, b, al, be)), rel=1e-10)
    hs1, su = cm.exascale_plot(n, p, 1, b, al, be, gamma)
    hsp, _ = cm.exascale_plot(n, p, p, b, al, be, gamma)
    assert close(hs1, su) and close(hsp, su)


@pytest.mark.parametrize("P,Q,I,J,b,B", [(16, 16, 4, 4, 64, 64), (16, 16, 4, 4, 64, 256),
                                         (8, 8, 2, 2, 32, 128), (32, 32, 1, 1, 64, 64)])
def test_grid_form_reduces_to_the_paper_on_square_grids(P, Q, I, J, b, B):
    n, p, G = 8192, P * Q, I * J
    for L, W, hs in ((cm.L_vdg, cm.W_vdg, cm.hsumma_vdg),
                     (cm.L_binomial, cm.W_binomial, cm.hsumma_binomial)):
        inner, outer = cm.comm_grid(n, P, Q, I, J, b, B, L, W, 2e-6, 1e-9)
        li, lo, bi, bo = hs(n, p, G, b, B, 2e-6, 1e-9)
        assert close(inner, li + bi) and close(outer, lo + bo)


@pytest.mark.parametrize("P,Q,I,J", [(4, 16, 2, 4), (6, 10, 3, 5), (2, 32, 1, 8), (12, 8, 4, 2)])
def test_grid_form_is_symmetric_under_transposition(P, Q, I, J):
    # swapping P <-> Q and I <-> J exchanges the roles of A and B (C^T = B^T A^T)
    n, b, B = 10000, 128, 512
    for L, W in ((cm.L_vdg, cm.W_vdg), (cm.L_binomial, cm.W_binomial)):
        a = cm.comm_grid(n, P, Q, I, J, b, B, L, W, 2e-6, 1e-9)
        t = cm.comm_grid(n, Q, P, J, I, b, B, L, W, 2e-6, 1e-9)
        assert close(a[0], t[0]) and close(a[1], t[1])
        # one group: nothing between groups; one process per group: nothing inside
        assert cm.comm_grid(n, P, Q, 1, 1, b, B, L, W, 2e-6, 1e-9)[1] == 0.0
        assert cm.comm_grid(n, P, Q, P, Q, b, B, L, W, 2e-6, 1e-9)[0] == 0.0


def test_levels_reduce_to_summa_and_hsumma():
    n, P, Q, b, B = 8192, 16, 8, 64, 256
    for L, W in ((cm.L_vdg, cm.W_vdg), (cm.L_binomial, cm.W_binomial)):
        one = cm.comm_levels(n, P, Q, [P], [Q], [b], L, W, 2e-6, 1e-9)
        assert close(sum(one), sum(cm.comm_grid(n, P, Q, 1, 1, b, b, L, W, 2e-6, 1e-9)))
        two = cm.comm_levels(n, P, Q, [4, P // 4], [2, Q // 2], [B, b], L, W, 2e-6, 1e-9)
        inner, outer = cm.comm_grid(n, P, Q, 4, 2, b, B, L, W, 2e-6, 1e-9)
        assert close(two[0], outer) and close(two[1], inner)
        # a level of one unit moves nothing
        three = cm.comm_levels(n, P, Q, [1, 4, P // 4], [1, 2, Q // 2], [1024, B, b], L, W,
                               2e-6, 1e-9)
        assert three[0] == 0.0 and close(three[1], outer) and close(three[2], inner)


@pytest.mark.parametrize("name", sorted(PLATFORMS))
def test_levels_closed_form(name):
    pf = PLATFORMS[name]
    n, p, b, al, be = pf["n"], pf["p"], pf["b"], pf["alpha"], pf["beta"]
    assert close(cm.levels_vdg(n, p, 1, b, al, be), sum(cm.summa_vdg(n, p, b, al, be)))
    assert close(cm.levels_vdg(n, p, 2, b, al, be), cm.optimal_vdg(n, p, b, al, be), rel=1e-11)
    # equal fan-out at every level on a grid where it is an integer
    for levels, q in ((3, 4), (2, 8), (4, 2)):
        P = q ** levels
        per = cm.comm_levels(n, P, P, [q] * levels, [q] * levels, [b] * levels,
                             cm.L_vdg, cm.W_vdg, al, be)
        assert close(sum(per), cm.levels_vdg(n, P * P, levels, b, al, be), rel=1e-11)
