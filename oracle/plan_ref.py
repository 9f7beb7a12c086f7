"""Reference of the processor grid, grouping, distribution and step schedule.

TEST INFRASTRUCTURE ONLY.  Written from Sec. II-A, Sec. III and Alg. 1 of the
paper; independent of the library's own plan code, which it is used to check.

Notation (paper -> here): the s x t processor grid is P x Q; its I x J
arrangement of groups has (P/I) x (Q/J) processors per group; processor
(i, j) of group (x, y) is grid processor (pr, pc) = (x*(P/I) + i, y*(Q/J) + j).
The outer block ("between groups") is M, the inner block b, with b <= M
(Sec. III); the paper's matrix dims (M, L, N) of Alg. 1 are m, k, n here.

Readings taken where the paper is silent or garbled:
  * G must factor as I*J with I | P and J | Q; among the factorizations the
    most square one is used (the analysis assumes sqrt(G) x sqrt(G) groups),
    ties broken by the smaller I.
  * Alg. 1 names the owner of A's pivot column by comparing row-group
    indices; a column of A is owned by a processor column, so the test is on
    the column-group index y and in-group column j (B symmetric with x, i).
  * Block distribution with P not dividing m: tile pr holds rows
    [floor(pr*m/P), floor((pr+1)*m/P)) (never empty when P <= m).
  * Block-cyclic distribution (named as future work): ScaLAPACK convention,
    block nb, first block on processor 0; global index g lives on processor
    (g div nb) mod P at local index (g div (nb*P))*nb + g mod nb.
  * A (m x k) is distributed like C by rows and its k columns over the Q
    processor columns; B (k x n) has its k rows over the P processor rows.
  * Outer step g covers k-columns [g*M, min((g+1)*M, k)); its inner steps
    split that range into pieces of b (the last one possibly shorter).

Pinned by tests/test_oracle.py: the Fig. 2 example (6 x 6 grid as 3 x 3
groups of 2 x 2, golden fixture), Fig. 4 (B/b inner steps per outer step),
the step identity n/B x B/b = n/b, and brute-force enumeration of the
distributions.
"""
from __future__ import annotations

from dataclasses import dataclass


def factor_groups(P: int, Q: int, G: int) -> tuple[int, int]:
    """(I, J) with I*J == G, I | P, J | Q; most square, then smaller I."""
    if P < 1 or Q < 1 or G < 1:
        raise ValueError("P, Q, G must be >= 1")
    best = None
    for I in range(1, P + 1):
        if P % I or G % I:
            continue
        J = G // I
        if J > Q or Q % J:
            continue
        key = (max(I, J) * 1.0 / min(I, J), I)
        if best is None or key < best[0]:
            best = (key, (I, J))
    if best is None:
        raise ValueError("G=%d cannot be arranged as I x J groups with I | %d, J | %d"
                         % (G, P, Q))
    return best[1]


def group_coords(pr: int, pc: int, P: int, Q: int, I: int, J: int):
    """(x, y, i, j): processor (pr, pc) is processor (i, j) of group (x, y)."""
    gp, gq = P // I, Q // J
    return pr // gp, pc // gq, pr % gp, pc % gq


# ------------------------------------------------------------ distributions

def block_range(length: int, parts: int, r: int) -> tuple[int, int]:
    return (r * length) // parts, ((r + 1) * length) // parts


def block_owner(g: int, length: int, parts: int) -> int:
    for r in range(parts):
        a, b = block_range(length, parts, r)
        if a <= g < b:
            return r
    raise IndexError(g)


def cyclic_owner(g: int, nb: int, parts: int) -> int:
    return (g // nb) % parts


def cyclic_local(g: int, nb: int, parts: int) -> int:
    return (g // (nb * parts)) * nb + g % nb


def cyclic_count(length: int, nb: int, parts: int, r: int) -> int:
    """Number of global indices of [0, length) owned by processor r."""
    return sum(1 for g in range(length) if cyclic_owner(g, nb, parts) == r)


def local_indices(length: int, parts: int, r: int, dist: str, nb: int) -> list[int]:
    """Global indices held by processor r, in local order."""
    if dist == "block":
        a, b = block_range(length, parts, r)
        return list(range(a, b))
    idx = [g for g in range(length) if cyclic_owner(g, nb, parts) == r]
    idx.sort(key=lambda g: cyclic_local(g, nb, parts))
    return idx


def owner(g: int, length: int, parts: int, dist: str, nb: int) -> int:
    if dist == "block":
        return block_owner(g, length, parts)
    return cyclic_owner(g, nb, parts)


def local_index(g: int, length: int, parts: int, dist: str, nb: int) -> int:
    if dist == "block":
        return g - block_range(length, parts, block_owner(g, length, parts))[0]
    return cyclic_local(g, nb, parts)


# ------------------------------------------------------------------ steps

@dataclass(frozen=True)
class Step:
    index: int      # global step number s
    outer: int      # outer step g
    inner: int      # inner step within g
    k0: int
    k1: int


def steps(k: int, b: int, M: int) -> list[Step]:
    """The two-level step schedule of Alg. 1 over the k dimension."""
    if b < 1 or M < b or M % b:
        raise ValueError("need 1 <= b <= M and b | M")
    out = []
    s = 0
    g = 0
    for g0 in range(0, k, M):
        g1 = min(g0 + M, k)
        t = 0
        for k0 in range(g0, g1, b):
            out.append(Step(s, g, t, k0, min(k0 + b, g1)))
            s += 1
            t += 1
        g += 1
    return out


def tile_shapes(m: int, n: int, P: int, Q: int, dist: str, nb: int):
    """{(pr, pc): (rows, cols)} of the local C tiles."""
    out = {}
    for pr in range(P):
        for pc in range(Q):
            out[(pr, pc)] = (len(local_indices(m, P, pr, dist, nb)),
                             len(local_indices(n, Q, pc, dist, nb)))
    return out
