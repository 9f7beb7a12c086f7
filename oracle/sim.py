"""Explicit simulation of Hierarchical SUMMA (Alg. 1) with per-processor memory.

TEST INFRASTRUCTURE ONLY.  Every virtual processor (pr, pc) owns its local
blocks of A, B and C (as the block or block-cyclic distribution assigns them,
see plan_ref) and receive buffers.  A "broadcast" copies a root's buffer into
the buffers of the other members of a communicator; a root can only send what
its own memory holds, so a wrong owner map shows up as NaN (unreceived) data or
as a wrong product.

Per outer step g (k-columns [g*M, ...)), following Alg. 1:
  1. each processor column that owns columns of A's outer panel copies them
     (Copy_Block_group) and broadcasts them among the processors holding the
     same in-group position in the other groups of the processor row
     (group_row_comm = {P(x,*)(i,j)}); B likewise along processor columns
     (group_col_comm = {P(*,y)(i,j)});
  2. for each inner step (b-wide piece), the processor of each group holding
     the piece selects it (Copy_Block_A/B) and broadcasts it inside its group
     (row_comm = {P(x,y)(i,*)}, col_comm = {P(x,y)(*,j)});
  3. each processor does C_loc += Block_A x Block_B (DGemm) with the plain
     k-ordered sum of core.gemm_view.

Because each local entry receives its products in increasing k, starting from
0, the gathered result equals core.gemm(A, B) bit for bit for any operands.
"""
from __future__ import annotations

import numpy as np

from . import core
from . import plan_ref as pr_


def hsumma(A, B, P: int, Q: int, G: int, b: int, M: int, dist: str = "block",
           nb: int | None = None, trace: list | None = None) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    m, k = A.shape
    n = B.shape[1]
    if B.shape[0] != k:
        raise ValueError("inner dimensions differ")
    if nb is None:
        nb = b
    I, J = pr_.factor_groups(P, Q, G)
    gp, gq = P // I, Q // J

    rows = {r: pr_.local_indices(m, P, r, dist, nb) for r in range(P)}
    cols = {c: pr_.local_indices(n, Q, c, dist, nb) for c in range(Q)}
    # k is split over Q (A's columns) and over P (B's rows).
    kA = {c: pr_.local_indices(k, Q, c, dist, nb) for c in range(Q)}
    kB = {r: pr_.local_indices(k, P, r, dist, nb) for r in range(P)}

    # Local memory of every processor.
    Aloc, Bloc, Cloc = {}, {}, {}
    for r in range(P):
        for c in range(Q):
            Aloc[r, c] = A[np.ix_(rows[r], kA[c])] if kA[c] else np.zeros((len(rows[r]), 0))
            Bloc[r, c] = B[np.ix_(kB[r], cols[c])] if kB[r] else np.zeros((0, len(cols[c])))
            Cloc[r, c] = np.zeros((len(rows[r]), len(cols[c])))

    for g, outer_steps in _outer_groups(pr_.steps(k, b, M)):
        g0, g1 = outer_steps[0].k0, outer_steps[-1].k1
        w = g1 - g0
        # Receive buffers for the outer panel, NaN until something arrives.
        BgA = {(r, c): np.full((len(rows[r]), w), np.nan) for r in range(P) for c in range(Q)}
        BgB = {(r, c): np.full((w, len(cols[c])), np.nan) for r in range(P) for c in range(Q)}

        # ---- step 1: broadcast between groups ------------------------------
        for kk in range(g0, g1):
            q = pr_.owner(kk, k, Q, dist, nb)            # processor column owning A(:, kk)
            lq = pr_.local_index(kk, k, Q, dist, nb)
            y_q, j_q = q // gq, q % gq                    # its group column, in-group column
            for r in range(P):
                root = (r, q)
                data = Aloc[root][:, lq]                  # Copy_Block_group on the owner
                for z in range(J):                        # group_row_comm of the root
                    BgA[r, z * gq + j_q][:, kk - g0] = data
                if trace is not None:
                    trace.append(("A-outer", g, kk, root))
            p = pr_.owner(kk, k, P, dist, nb)            # processor row owning B(kk, :)
            lp = pr_.local_index(kk, k, P, dist, nb)
            x_p, i_p = p // gp, p % gp
            for c in range(Q):
                root = (p, c)
                data = Bloc[root][lp, :]
                for z in range(I):                        # group_col_comm of the root
                    BgB[z * gp + i_p, c][kk - g0, :] = data
                if trace is not None:
                    trace.append(("B-outer", g, kk, root))

        # ---- step 2 + 3: inner steps inside each group ---------------------
        for st in outer_steps:
            wi = st.k1 - st.k0
            BA = {(r, c): np.full((len(rows[r]), wi), np.nan) for r in range(P) for c in range(Q)}
            BB = {(r, c): np.full((wi, len(cols[c])), np.nan) for r in range(P) for c in range(Q)}
            for kk in range(st.k0, st.k1):
                q = pr_.owner(kk, k, Q, dist, nb)
                j_q = q % gq
                for r in range(P):
                    for y in range(J):
                        root = (r, y * gq + j_q)          # holds the piece inside group column y
                        data = BgA[root][:, kk - g0]      # Copy_Block_A
                        for c in range(gq):               # row_comm inside the group
                            BA[r, y * gq + c][:, kk - st.k0] = data
                p = pr_.owner(kk, k, P, dist, nb)
                i_p = p % gp
                for c in range(Q):
                    for x in range(I):
                        root = (x * gp + i_p, c)
                        data = BgB[root][kk - g0, :]      # Copy_Block_B
                        for r in range(gp):               # col_comm inside the group
                            BB[x * gp + r, c][kk - st.k0, :] = data
            for r in range(P):
                for c in range(Q):
                    if Cloc[r, c].size and wi:
                        core.gemm_view(np.ascontiguousarray(BA[r, c]),
                                       np.ascontiguousarray(BB[r, c]), Cloc[r, c])

    C = np.full((m, n), np.nan)
    for r in range(P):
        for c in range(Q):
            if rows[r] and cols[c]:
                C[np.ix_(rows[r], cols[c])] = Cloc[r, c]
    return C


def _outer_groups(step_list):
    cur, acc = None, []
    for st in step_list:
        if cur is not None and st.outer != cur:
            yield cur, acc
            acc = []
        cur = st.outer
        acc.append(st)
    if acc:
        yield cur, acc
