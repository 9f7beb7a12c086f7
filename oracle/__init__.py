"""CPU oracle for the Hierarchical SUMMA local update -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU
library (``paper_1306_4161_amd``): it neither imports it nor is imported by
it.  Both sides receive the same operands from the seeded generators in
``paper_1306_4161_amd.inputs``, which hold none of the method's arithmetic.

Modules
  core      ctypes binding of ``oracle.c`` (plain triple loop, Dot2,
            sampled entries, Freivalds' check) and exact rational brute force.
  plan_ref  the processor grid, its grouping, the block and block-cyclic
            distributions and the step schedule, written from Sec. III and
            Alg. 1 of the paper.
  sim       an explicit simulation of Alg. 1: per-processor buffers and
            copy-based broadcasts, local update by ``core.gemm``.
  split_ref the operand-splitting rule of the precision form (an
            Ozaki-style error-free split; not in the paper) and the exact
            value of the truncated split product.
  mlp_ref   float64 forward/backward of the small cost-model network.
  lu_ref    LU factorisation without pivoting by textbook elimination (the
            workload whose trailing update is the local update).

Parity status per function is stated in each module header.
"""
