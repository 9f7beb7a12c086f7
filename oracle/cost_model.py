"""Reference of the paper's communication-cost model (Sec. IV).

TEST INFRASTRUCTURE ONLY.  Written from Sec. IV of the paper (Hockney's
point-to-point model, the binomial-tree and Van de Geijn broadcasts, the
SUMMA and HSUMMA costs of Sec. IV-A/IV-B and Tables I-II, the general
broadcast model of eq. (1)-(5), the derivative of eq. (10), the condition of
eq. (11) and the optimum of eq. (12)); independent of the library's own
model code, which it is used to check.

Notation as in the paper: n x n matrices on a sqrt(p) x sqrt(p) grid, G
groups arranged sqrt(G) x sqrt(G), inner block b, outer block B; alpha the
latency, beta the reciprocal bandwidth (seconds per matrix element), gamma
the time of one floating-point operation.  Every cost is in seconds.

Readings (the paper is silent or garbled):
  * Message sizes are counted in matrix elements, as the paper's own
    derivations do (n b / sqrt(p) elements per broadcast).
  * The computation cost 2 n^3 / p of Tables I-II is in floating-point
    operations; its time is that count times gamma.
  * The row and column broadcasts of one step are counted as two
    broadcasts (the factor 2 of eq. (2)), as every closed form of the
    paper does.
  * For a grid that is not square (P x Q processes, I x J groups) the same
    reasoning gives: A's pivot column block goes to the Q processes of a row
    (n b / P elements each), B's pivot row block to the P processes of a
    column (n b / Q each); between groups the same happens over J (rows) and
    I (columns) groups with the outer block B, inside a group over Q / J and
    P / I processes with b.  It reduces to eq. (2)-(5) for P = Q, I = J.

Functions
  bcast_binomial(m, p, alpha, beta), bcast_vdg(m, p, alpha, beta)
  L_binomial, W_binomial, L_vdg, W_vdg       L(p), W(p) of eq. (1)
  summa_binomial(n, p, b, alpha, beta)       Sec. IV-A, first item
  summa_vdg(n, p, b, alpha, beta)            Sec. IV-A, second item
  hsumma_binomial(n, p, G, b, B, alpha, beta)   inner + outer, Sec. IV-B
  hsumma_vdg(n, p, G, b, B, alpha, beta)
  T_S(n, p, b, L, W, alpha, beta)            eq. (2)
  T_HS(n, p, G, b, L, W, alpha, beta)        eq. (3)-(5), b = B
  dTHS_dG_vdg(n, p, G, b, alpha, beta)       eq. (10)
  minimum_at_sqrt_p(n, p, b, alpha, beta)    eq. (11)
  optimal_vdg(n, p, b, alpha, beta)          eq. (12)
  comm_grid(n, P, Q, I, J, b, B, L, W, alpha, beta)   the non-square reading
  exascale_plot(n, p, G, b, alpha, beta, gamma)   the curves of Fig. 10
  comm_levels(n, P, Q, Is, Js, blocks, L, W, alpha, beta)   more than two levels
  levels_vdg(n, p, levels, b, alpha, beta)   their equal-fan-out closed form
"""
from __future__ import annotations

import math


def log2(x: float) -> float:
    return math.log(x, 2)


# -- broadcasts of m elements among p processes (Sec. IV) --------------------

def bcast_binomial(m, p, alpha, beta):
    return log2(p) * (alpha + m * beta)


def bcast_vdg(m, p, alpha, beta):
    return (log2(p) + p - 1) * alpha + 2 * (p - 1) / p * m * beta


# the same two algorithms in the form T = L(p) alpha + m W(p) beta of eq. (1)
def L_binomial(p):
    return log2(p)


def W_binomial(p):
    return log2(p)


def L_vdg(p):
    return log2(p) + p - 1


def W_vdg(p):
    return 2 * (p - 1) / p


# -- SUMMA (Sec. IV-A), returns (latency seconds, bandwidth seconds) ----------

def summa_binomial(n, p, b, alpha, beta):
    return (log2(p) * alpha * n / b, log2(p) * beta * n * n / math.sqrt(p))


def summa_vdg(n, p, b, alpha, beta):
    sp = math.sqrt(p)
    return ((log2(p) + 2 * (sp - 1)) * alpha * n / b,
            4 * (1 - 1 / sp) * n * n / sp * beta)


# -- HSUMMA (Sec. IV-B): inner (inside groups) and outer (between groups) ----
# returns (latency inner, latency outer, bandwidth inner, bandwidth outer)

def hsumma_binomial(n, p, G, b, B, alpha, beta):
    sp = math.sqrt(p)
    return (log2(p / G) * alpha * n / b,
            log2(G) * alpha * n / B,
            log2(p / G) * beta * n * n / sp,
            log2(G) * beta * n * n / sp)


def hsumma_vdg(n, p, G, b, B, alpha, beta):
    sp, sg = math.sqrt(p), math.sqrt(G)
    return ((log2(p / G) + 2 * (sp / sg - 1)) * alpha * n / b,
            (log2(G) + 2 * (sg - 1)) * alpha * n / B,
            4 * (1 - sg / sp) * n * n / sp * beta,
            4 * (1 - 1 / sg) * n * n / sp * beta)


# -- general broadcast model, eq. (2)-(5) (b = B) ----------------------------

def T_S(n, p, b, L, W, alpha, beta):
    sp = math.sqrt(p)
    return 2 * (n / b * L(sp) * alpha + n * n / sp * W(sp) * beta)


def T_HS(n, p, G, b, L, W, alpha, beta):
    sp, sg = math.sqrt(p), math.sqrt(G)
    lat = 2 * n / b * (L(sg) + L(sp / sg)) * alpha
    band = 2 * n * n / sp * (W(sg) + W(sp / sg)) * beta
    return lat + band


def dTHS_dG_vdg(n, p, G, b, alpha, beta):
    """Eq. (10): derivative of the Van de Geijn HSUMMA cost in G (b = B)."""
    return (G - math.sqrt(p)) / (G * math.sqrt(G)) * (n * alpha / b - 2 * n * n / p * beta)


def minimum_at_sqrt_p(n, p, b, alpha, beta):
    """Eq. (11): G = sqrt(p) is the minimum in (1, p) iff alpha/beta > 2 n b / p."""
    return alpha / beta > 2 * n * b / p


def optimal_vdg(n, p, b, alpha, beta):
    """Eq. (12): Van de Geijn HSUMMA cost at G = sqrt(p), b = B."""
    q = p ** 0.25
    return (log2(p) + 4 * (q - 1)) * n / b * alpha + 8 * (1 - 1 / q) * n * n / math.sqrt(p) * beta


# -- the non-square reading --------------------------------------------------

def comm_grid(n, P, Q, I, J, b, B, L, W, alpha, beta):
    """(inner seconds, outer seconds) on a P x Q grid with I x J groups."""
    def bc(m, q):                      # eq. (1); L(1) = W(1) = 0
        return L(q) * alpha + m * W(q) * beta
    inner = n / b * (bc(n * b / P, Q / J) + bc(n * b / Q, P / I))
    outer = n / B * (bc(n * B / P, J) + bc(n * B / Q, I))
    return inner, outer


# -- Fig. 10 (exascale prediction), as its curves are printed ---------------

def exascale_plot(n, p, G, b, alpha, beta, gamma):
    """(HSUMMA, SUMMA) execution times of the two curves of Fig. 10."""
    comp = 2 * n ** 3 * gamma / p
    hs = comp + (n / b) * (log2(p) + 2 * (math.sqrt(p) / math.sqrt(G) + math.sqrt(G) - 2)) * alpha \
        + 4 * (n * n / math.sqrt(p)) * (2 - math.sqrt(G) / math.sqrt(p) - 1 / math.sqrt(G)) * beta
    su = comp + (n / b) * (log2(p) + 2 * (math.sqrt(p) - 1)) * alpha \
        + 4 * (n * n / math.sqrt(p)) * (1 - 1 / math.sqrt(p)) * beta
    return hs, su


# -- more than two levels (the paper's future work, Sec. VI) -----------------
# Level 0 is the outermost.  Level l arranges its units I_l x J_l (the
# products over the levels are P and Q) and moves blocks of width B_l
# (non-increasing, the innermost being b): every B_l-step broadcasts A's
# n B_l / P elements per process along J_l units of a row and B's n B_l / Q
# along I_l units of a column.  Two levels (I, J), (P/I, Q/J) with (B, b)
# are HSUMMA; one level (P, Q) with b is SUMMA.

def comm_levels(n, P, Q, Is, Js, blocks, L, W, alpha, beta):
    """Seconds of every level's broadcasts, outermost first."""
    out = []
    for I, J, Bl in zip(Is, Js, blocks):
        row = L(J) * alpha + n * Bl / P * W(J) * beta
        col = L(I) * alpha + n * Bl / Q * W(I) * beta
        out.append(n / Bl * (row + col))
    return out


def levels_vdg(n, p, levels, b, alpha, beta):
    """Van de Geijn cost with `levels` levels of equal fan-out p^(1/(2 levels))
    per dimension on a sqrt(p) x sqrt(p) grid, b at every level; levels = 1
    is SUMMA (Table II), levels = 2 the optimum of eq. (12)."""
    q = p ** (1.0 / (2 * levels))
    return ((log2(p) + 2 * levels * (q - 1)) * n / b * alpha
            + 4 * levels * (1 - 1 / q) * n * n / math.sqrt(p) * beta)
