/*
 * hsumma.h -- C ABI of the Hierarchical SUMMA local-update library (gfx950).
 *
 * The method (Quintin, Hasanov, Lastovetsky, "Hierarchical Parallel Matrix
 * Multiplication on Large-Scale Distributed Memory Platforms"): C = A x B on a
 * virtual P x Q processor grid (the paper's s x t, Sec. II-A), arranged as
 * I x J groups of (P/I) x (Q/J) processors (Sec. III).  The k dimension is
 * consumed in outer blocks of width M (the paper's B, "between groups") and
 * inner blocks of width b <= M ("inside a group"); every processor performs
 * the local update  C_loc += A_panel x B_panel  once per inner block
 * (Alg. 1, the DGemm call; Sec. II-A for the update rule c_ij += a_ik b_kj).
 *
 * On one GPU every virtual processor is a set of workgroups: its tile of C
 * is cut into macro-tiles, the processors of one group are steered to one
 * XCD (one L2), and the two broadcast levels become staging of the outer
 * panel and LDS streaming of the inner b-slices.  C is held in MFMA
 * accumulators across all inner steps of one outer step.
 *
 * Layout.  A is m x k, B is k x n, C is m x n, all row-major FP64 in device
 * memory with leading dimensions lda >= k, ldb >= n, ldc >= m's row length n
 * (elements).  Tiles are views of the global matrices: with the block
 * distribution a tile is a contiguous sub-block; with the block-cyclic one
 * it is the set of distribution blocks the processor owns.  Column-major
 * callers pass transposed problems.
 *
 * Ownership.  The caller owns A, B, C and the workspace `ws`: device memory
 * of at least hsumma_workspace_size() bytes, 256-byte aligned, required by
 * every compute call of every precision.  4 KiB alignment is recommended:
 * the split forms' digit planes start on 4 KiB boundaries of `ws`, and their
 * product kernels ran 1-2 % slower with planes 256 or 1536 bytes off such a
 * boundary in device memory.  The library allocates no device
 * memory and copies nothing from the host to the device: each compute call
 * first writes the plan's work-item table (the macro-tiles of every virtual
 * processor, see hsumma_work_items) into `ws` with a small kernel, then
 * launches the update kernels, which read their operands and the workspace
 * only.  A plan is a host object; a HIP graph it captures (opts.use_graph)
 * and the second stream and events of a split-form plan with look-ahead
 * (opts.lookahead) are owned by the plan and released by
 * hsumma_plan_destroy().  A, B, C and
 * `ws` must be ordinary (coarse-grained) device memory of the current
 * device: the split forms add into C with FP64 atomic adds, which need it.
 *
 * Streams and synchronisation.  `stream` is a hipStream_t passed as void*
 * (NULL = the null stream).  All compute calls are asynchronous on it and
 * never synchronise the device or the host; only hsumma_panel_slices waits
 * for `stream`.  hsumma_run of a look-ahead plan also launches on the
 * plan's own stream, ordered by events after the work already queued on
 * `stream`, and makes `stream` wait for all of it before the call's last
 * launch, so the call still ends on `stream`.  A, B, C and ws must not overlap.  Calls that share a
 * workspace must be ordered (one stream, or events).
 *
 * Non-finite inputs.  The FP64 path follows IEEE arithmetic (an Inf or NaN
 * in A or B reaches the entries of C whose sums include it).  The split
 * forms detect Inf and NaN in a panel and compute that panel with the FP64
 * kernel instead, so they propagate the same way.
 *
 * Errors.  Every int-returning call returns an hsumma_status.  Invalid
 * arguments return HSUMMA_ERR_INVALID (nothing is launched); HIP failures
 * return HSUMMA_ERR_DEVICE.  hsumma_last_error() gives a message for the
 * last failure on the calling thread.  The library never aborts.
 */
#ifndef HSUMMA_H
#define HSUMMA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hsumma_plan_s* hsumma_plan_t;

typedef enum {
  HSUMMA_OK = 0,
  HSUMMA_ERR_INVALID = -1,      /* bad argument or unsupported shape */
  HSUMMA_ERR_UNSUPPORTED = -2,  /* option not compiled in or not supported by the device */
  HSUMMA_ERR_DEVICE = -3,       /* a HIP call failed (message has its text) */
  HSUMMA_ERR_WORKSPACE = -4     /* workspace missing or too small */
} hsumma_status;

typedef enum {
  HSUMMA_FP64 = 0,         /* FP64 MFMA local update */
  HSUMMA_SPLIT_BF16 = 1,   /* digit split into BF16 slices, FP32-exact MFMA, FP64 recombination */
  HSUMMA_SPLIT_FP8 = 2,    /* the same with FP8-e4m3 slices */
  HSUMMA_SPLIT_INT8 = 3    /* the same with INT8 slices, INT32-exact MFMA (32 k per
                              instruction, twice the BF16 rate); M <= 8192 */
} hsumma_precision;

typedef enum {
  HSUMMA_DIST_BLOCK = 0,         /* block-checkerboard distribution (Sec. II-A, Sec. III) */
  HSUMMA_DIST_BLOCK_CYCLIC = 1   /* block-cyclic distribution (named as future work, Sec. VI) */
} hsumma_dist;

typedef struct {
  int64_t m;          /* rows of A and C; 0 => n                                */
  int64_t k;          /* columns of A = rows of B; 0 => n (Alg. 1's (M, L, N))  */
  int32_t dist;       /* hsumma_dist                                            */
  int32_t prec;       /* hsumma_precision                                       */
  int64_t nb;         /* block-cyclic block size; 0 => b                        */
  int32_t slices;     /* split forms: digits per operand, 0 => chosen per panel */
  int32_t min_slices; /* bounds of the per-panel choice; 0 => 3                 */
  int32_t max_slices; /*                     0 => 7 (BF16, FP8) or 8 (INT8)    */
  int32_t tile_m;     /* macro-tile rows;  0 => default / tuned                 */
  int32_t tile_n;     /* macro-tile cols;  0 => default / tuned                 */
  int32_t kc;         /* k-chunk staged per LDS buffer; 0 => default            */
  int32_t persistent; /* 1: one grouped persistent launch per step              */
  int32_t use_graph;  /* 1: hsumma_run replays a captured HIP graph             */
  int32_t tau_bits;   /* split forms, per-panel slice choice: the smallest s    */
                      /* whose modelled max error relative to (|A||B|)_ij is    */
                      /* <= 2^-tau_bits (model: bits(s) against the panel's     */
                      /* value spread and k, with random-sign cancellation over */
                      /* k credited only when no line repeats its low-order     */
                      /* bits; max_slices when the spread statistic is          */
                      /* saturated by a narrow panel); a panel needing more     */
                      /* than max_slices goes to the FP64 kernel;               */
                      /* 0 => 48 (50 for INT8)                                  */
  int32_t staged;     /* FP64 path: 1 = always the register-staged kernel,      */
                      /* 0 = direct-to-LDS loads where alignment allows         */
  int32_t waves;      /* FP64 path: waves per workgroup of the macro-tile's     */
                      /* kernel; 0 => the tile's first compiled configuration   */
  int32_t lookahead;  /* hsumma_lu: nonzero = factor the next panel while the  */
                      /* rest of the trailing update runs on a second stream.   */
                      /* Split forms: 1 = hsumma_run splits outer panel g + 1   */
                      /* on a second stream while the products of panel g run   */
                      /* (the workspace holds two sets of digit planes; panel g */
                      /* uses set g % 2 in every call); 2 = the same, but the   */
                      /* overlap is used only where one product launch has      */
                      /* fewer work items than the device has CUs (where it     */
                      /* pays; elsewhere the plain sequence runs).  Same        */
                      /* result, bit for bit.  No effect on the FP64 path;      */
                      /* other values are invalid                               */
  int32_t wgs_per_cu; /* persistent launches: workgroups per CU, at most what   */
                      /* fits; 0 => what fits.  Fewer leave room on every CU    */
                      /* for concurrent work (hsumma_lu's look-ahead)           */
  int32_t reserved[1];
} hsumma_opts;

/* Fill *o with defaults (all zero: square, block, FP64, default tiles). */
void hsumma_opts_default(hsumma_opts* o);

/*
 * Build a plan for C = A x B with A m x k, B k x n (m, k from opts, else n).
 * P x Q grid (P <= m, Q <= n), G groups (Sec. III: G = I*J with I | P and
 * J | Q; the most square arrangement is chosen), inner block b >= 1, outer
 * block M with b <= M (Sec. III) and M a multiple of b.  G = 1 or G = P*Q is
 * plain SUMMA (Sec. III).  m, n and k must be below 2^31.  Host only:
 * validates, builds the step schedule and the work-item table.  Returns
 * HSUMMA_ERR_INVALID on bad input.
 */
int hsumma_plan(hsumma_plan_t* out, int64_t n, int32_t P, int32_t Q, int32_t G,
                int64_t b, int64_t M, const hsumma_opts* opts);
void hsumma_plan_destroy(hsumma_plan_t plan);

/* Queries (host only). */
/* Bytes of device workspace every compute call needs (> 0). */
int hsumma_workspace_size(hsumma_plan_t plan, size_t* bytes);
/* Inner steps (Sec. III: k/b steps of width b, the k/M outer blocks each
 * split into M/b): the sum over outer blocks of ceil(width/b), so a ragged
 * last block of k gives a shorter last step. */
int hsumma_num_steps(hsumma_plan_t plan, int64_t* steps);
int hsumma_num_outer_steps(hsumma_plan_t plan, int64_t* steps);    /* ceil(k/M), Sec. III */
int hsumma_groups(hsumma_plan_t plan, int32_t* I, int32_t* J);     /* Sec. III arrangement */
/* Rows and columns of C owned by processor (pr, pc) (Sec. II-A: processor
 * (i, j) owns one block of C; the block-cyclic distribution of Sec. VI owns
 * every P-th (Q-th) block of nb rows (columns) starting at pr (pc)). */
int hsumma_tile_shape(hsumma_plan_t plan, int32_t pr, int32_t pc,
                      int64_t* m_loc, int64_t* n_loc);
/*
 * Step s of the schedule (Alg. 1): its k-range [k0, k1), outer step, and the
 * owners of its panels: processor column q owning A(:, k0) and processor row
 * p owning B(k0, :), with their group index and in-group index (the pivot
 * functions of Alg. 1).
 */
int hsumma_step_info(hsumma_plan_t plan, int64_t s, int64_t* k0, int64_t* k1,
                     int64_t* outer, int32_t* owner_col, int32_t* owner_row,
                     int32_t* group_col, int32_t* group_row,
                     int32_t* in_group_col, int32_t* in_group_row);
/* Number of work items (macro-tiles over all tiles) per launch. */
int hsumma_num_items(hsumma_plan_t plan, int64_t* items);
/*
 * The macro-tile the plan's update kernels use: rows, columns, k-chunk and
 * waves per workgroup (the split forms: 64 x 128, 16-k steps or 32-k for
 * INT8, 4 waves).  With no tile option given, the FP64 path takes 32 x 32
 * when fewer than 768 macro-tiles of 64 x 64 would make a launch; 64 x 64
 * when a processor's tile is under 512 on a side (m/P or n/Q), the outer
 * block M is under 128, or fewer than 4096 macro-tiles of 128 x 128 would
 * make a launch; 128 x 64 when M >= 1024; else 128 x 128 (fitted to the
 * autotuner's timings of 2013 shapes).
 */
int hsumma_tile_config(hsumma_plan_t plan, int32_t* tile_m, int32_t* tile_n, int32_t* kc,
                       int32_t* waves);
/*
 * The work-item table the compute calls write into the workspace, as the
 * plan defines it (host memory, out has 4 x hsumma_num_items() int32):
 * item t is rows [r0, r0 + h) and columns [c0, c0 + w) of C, stored as
 * out[4t .. 4t+3] = r0, c0, h, w.  Items are listed group by group (Sec.
 * III), processor by processor inside a group and macro-tile by macro-tile
 * inside a processor's tile (Sec. II-A), cut into 8 equal consecutive
 * lists (one per XCD); in the persistent mode and the split forms each list
 * is in decreasing order of area (stable).
 */
int hsumma_work_items(hsumma_plan_t plan, int32_t* out, int64_t capacity);
/*
 * Write the work-item table into the workspace (bytes [0, 16 x items) of
 * ws, the layout of hsumma_work_items), as every compute call does first.
 * Asynchronous on `stream`.
 */
int hsumma_prepare_workspace(hsumma_plan_t plan, void* ws, size_t ws_bytes, void* stream);

/*
 * One inner step s (0 <= s < num_steps): for every tile,
 *   C_loc += A(rows, k0:k1) x B(k0:k1, cols)          (Alg. 1, DGemm)
 * i.e. C += A(:, k0:k1) B(k0:k1, :).  Accumulates into C as given.
 */
int hsumma_local_update(hsumma_plan_t plan, int64_t step,
                        const double* A, int64_t lda, const double* B, int64_t ldb,
                        double* C, int64_t ldc, void* ws, size_t ws_bytes, void* stream);

/*
 * One outer step g (Sec. III: the between-group step of width M): all inner
 * steps of the outer block in one launch, C held in registers across them.
 * Accumulates into C.  FP64 path: bitwise equal to the sequence of its
 * hsumma_local_update calls (the MFMA k-groups restart at every inner-step
 * boundary).  Split forms: the outer step splits its M-wide panel once,
 * while each hsumma_local_update splits its own b-wide panel, so the two
 * truncate differently (each is the truncated product of its own panels).
 */
int hsumma_outer_update(hsumma_plan_t plan, int64_t outer,
                        const double* A, int64_t lda, const double* B, int64_t ldb,
                        double* C, int64_t ldc, void* ws, size_t ws_bytes, void* stream);

/*
 * Split forms only: the slice-product launch of outer step g alone, on the
 * digit planes the workspace holds from a previous call that split that
 * outer step's panel (C += its product; with look-ahead, set g % 2 of the
 * planes); a panel that split sent to the
 * FP64 kernel (slice count 0) is recomputed by it from A and B.  Lets a
 * caller time or repeat the matrix-core part without the split.
 */
int hsumma_outer_products(hsumma_plan_t plan, int64_t outer, const double* A, int64_t lda,
                          const double* B, int64_t ldb, double* C, int64_t ldc, void* ws,
                          size_t ws_bytes, void* stream);

/*
 * The whole product C = A x B (Alg. 1: every outer step of width M, each of
 * M/b inner steps; Sec. II-A: c_ij = sum_k a_ik b_kj once all steps are
 * done): every outer step in order, the first one storing instead of
 * accumulating, so C needs no clearing.  With
 * opts.use_graph the launch sequence (work-item table included) is captured
 * once per (pointers, stream, device) and replayed.  With opts.lookahead (a
 * split form, more than one outer step) the split of each next panel runs
 * on a stream the plan creates on its first such call (Sec. VI: the next
 * step's panel work overlaps this step's update); events order it, and the
 * call's work all ends on `stream`.  Such a plan then serves one device, and
 * its calls are serialised on the host (they share that stream).
 */
int hsumma_run(hsumma_plan_t plan, const double* A, int64_t lda, const double* B,
               int64_t ldb, double* C, int64_t ldc, void* ws, size_t ws_bytes,
               void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as hsumma_run, with the workspace taken from a scratch array the
 * library holds in device memory (hsumma_noalloc_max_workspace() bytes per
 * device, held from the library's load on that device until the process
 * ends).  The call allocates nothing and takes no workspace argument; it
 * always launches directly (opts.use_graph is ignored: instantiating a graph
 * may allocate).  A plan whose hsumma_workspace_size() exceeds the scratch
 * array is rejected with HSUMMA_ERR_WORKSPACE before anything is launched.
 * Every such call on one device uses that device's one array: calls that
 * overlap on a device (other streams, other threads) race and must be
 * ordered by the caller.  Each call rewrites or clears everything it reads
 * there, so results do not depend on earlier calls.
 */
int hsumma_run_noalloc(hsumma_plan_t plan, const double* A, int64_t lda, const double* B,
                       int64_t ldb, double* C, int64_t ldc, void* stream);
/* Bytes of the scratch array behind hsumma_run_noalloc (64 MiB). */
size_t hsumma_noalloc_max_workspace(void);

/* Slice count chosen for each outer panel by the last split-form call
 * (copied to host; synchronises `stream`).  counts has num_outer_steps room.
 * A count of 0 means the panel was computed by the FP64 kernel: it held an
 * Inf or a NaN, or (automatic count) the slice-count model needed more than
 * max_slices digits for an error within 2^-tau_bits of (|A||B|)_ij. */
int hsumma_panel_slices(hsumma_plan_t plan, const void* ws, int32_t* counts, void* stream);

/*
 * Layout of the split forms' workspace after a call: byte offsets of the A
 * digit planes (planes x m x Wp digits, 2 B per BF16 digit or 1 B per
 * FP8-e4m3 or INT8 digit, stored k16-block-major: digit (plane, row, k) at
 * plane*m*Wp + (k/16)*m*16 + row*16 + k%16; INT8 k32-block-major, at
 * plane*m*Wp + (k/32)*m*32 + row*32 + k%32), the B digit planes (the same
 * with n columns: B transposed), the int32 row exponents of A and column
 * exponents of B.  They hold the most recently split panel (with look-ahead:
 * the most recently split even outer panel; odd ones use a second set); of
 * its planes only the first s (its slice count, see hsumma_panel_slices)
 * are written.
 * Lets a caller inspect the split; HSUMMA_ERR_UNSUPPORTED for the FP64
 * path.
 */
int hsumma_split_layout(hsumma_plan_t plan, size_t* off_digA, size_t* off_digB,
                        size_t* off_eA, size_t* off_fB, int32_t* Wp, int32_t* planes);

/*
 * Self-test of the matrix-core accumulation the split forms rely on:
 * d (32 x 32 FP32, row-major) = a (32 x k digits, row-major) x b (k x 32
 * digits, row-major) by chained 32x32x16 MFMAs (the slice kernels'
 * instructions) with FP32 accumulation, fmt 0 = BF16 bit patterns (2 B),
 * 1 = FP8-e4m3 bytes; fmt 2 = INT8 bytes by 32x32x32 MFMAs with INT32
 * accumulation, returned converted to FP32.  k a positive multiple of 16
 * (32 for INT8).  Integer digits whose partial sums stay within 2^24 must
 * come back exact.  All pointers are device memory; asynchronous on
 * `stream`.
 */
int hsumma_mfma_exact_probe(int32_t fmt, const void* a, const void* b, int32_t k, float* d,
                            void* stream);

/*
 * LU factorisation without pivoting, A = L U in place, with the trailing-
 * matrix update done by the HSUMMA local update (Sec. VI names LU as a
 * workload for the hierarchical panel updates; the trailing update A22 -=
 * L21 U12 is the update C += A_panel x B_panel of Sec. II-A).  Blocked with
 * the two block sizes of Sec. III: outer panels of M columns factored in
 * inner blocks of b <= 64 columns (M a multiple of b); after each outer
 * panel the trailing matrix takes one HSUMMA outer update with k = M on the
 * P x Q grid with G groups (clamped to the trailing block's size), in the
 * precision of opts.prec (FP64 or a split form).  L (unit lower, without its
 * diagonal) and U overwrite A (row-major, n x n, leading dimension lda >= n).
 * No pivoting: the caller guarantees nonzero leading principal minors (e.g.
 * a diagonally dominant matrix); a zero pivot yields Inf or NaN in the
 * factors.  The plan is host memory; ws (hsumma_lu_workspace_size() bytes,
 * 256-byte aligned, 4 KiB recommended as for hsumma_run) holds the negated panel L21 (n x M doubles) and the
 * trailing updates' workspace.  Asynchronous on `stream`.
 *
 * opts.lookahead = 1 overlaps the factorisation of each outer panel with the
 * previous trailing update (the overlap of panel work and computation the
 * paper names as future work, Sec. VI): the trailing update is split into
 * the next panel's block rows and columns, done first on `stream`, and the
 * rest, done on a second stream while the next panel is factored on
 * `stream`; the L21 panel is double-buffered (two n x M buffers in ws).  The
 * plan then creates one non-blocking HIP stream and two events on its first
 * hsumma_lu call (on that device; hsumma_lu_plan_destroy releases them), and
 * every later call must be on the same device.  The concurrent part is a
 * persistent launch of opts.wgs_per_cu workgroups per CU (0 => 1), which
 * leaves room on every CU for the panel kernels.  FP64: the results are the
 * same bits as without look-ahead (every entry sums the same products in the
 * same order).  Split forms: each block of the trailing update takes its own
 * slice count, so results may differ within the split's error bound.
 * hsumma_lu returns once all work is ordered before `stream`'s next command.
 */
typedef struct hsumma_lu_plan_s* hsumma_lu_plan_t;
int hsumma_lu_plan(hsumma_lu_plan_t* out, int64_t n, int32_t P, int32_t Q, int32_t G, int64_t b,
                   int64_t M, const hsumma_opts* opts);
int hsumma_lu_workspace_size(hsumma_lu_plan_t plan, size_t* bytes);
int hsumma_lu(hsumma_lu_plan_t plan, double* A, int64_t lda, void* ws, size_t ws_bytes,
              void* stream);
void hsumma_lu_plan_destroy(hsumma_lu_plan_t plan);

/*
 * Communication-cost model of the distributed algorithm (Sec. IV) and the
 * choice of G it implies.  Host only (no device work, no allocation).
 *
 * Hockney's model: one message of m elements between two processes costs
 * alpha + m beta; gamma is the time of one floating-point operation on one
 * process.  Broadcasts of m elements among q processes (Sec. IV):
 *   HSUMMA_BCAST_BINOMIAL      log2(q) (alpha + m beta)
 *   HSUMMA_BCAST_VAN_DE_GEIJN  (log2(q) + q - 1) alpha + 2 (q - 1)/q m beta
 * On a P x Q grid with G = I x J groups (the plan's most square
 * arrangement), n x n matrices, inner block b and outer block B: every inner
 * step broadcasts A's pivot block (n b / P elements per process) along a
 * process row inside the group (Q / J processes) and B's (n b / Q) along a
 * process column (P / I); every outer step does the same between groups (J
 * and I groups) with B.  For P = Q = sqrt(p) and I = J = sqrt(G) these are
 * the costs of Sec. IV-A/IV-B and Tables I-II (eq. (2)-(5) when b = B); G = 1
 * (or G = P Q with b = B) is SUMMA.  Message sizes are in elements.
 */
typedef enum { HSUMMA_BCAST_BINOMIAL = 0, HSUMMA_BCAST_VAN_DE_GEIJN = 1 } hsumma_bcast;

typedef struct {
  double alpha;   /* seconds per message (latency)                              */
  double beta;    /* seconds per matrix element (reciprocal bandwidth)          */
  double gamma;   /* seconds per floating-point operation on one process        */
} hsumma_platform;

typedef struct {
  double comp;             /* 2 n^3 / (P Q) operations x gamma (Tables I-II)      */
  double latency_inner;    /* alpha terms of the broadcasts inside groups         */
  double latency_outer;    /* alpha terms of the broadcasts between groups        */
  double bandwidth_inner;  /* beta terms inside groups                            */
  double bandwidth_outer;  /* beta terms between groups                           */
  double comm;             /* the four terms added                                */
  double total;            /* comp + comm (no overlap, as in the paper)           */
} hsumma_cost;

/* Time of one broadcast of m elements among q >= 1 processes. */
int hsumma_model_bcast(int32_t algo, const hsumma_platform* pf, double m, double q,
                       double* seconds);
/* Cost of C = A x B (n x n) on a P x Q grid with G groups.  Returns
 * HSUMMA_ERR_INVALID if G cannot be arranged as I x J with I | P, J | Q, or
 * if a size is not positive or b > B. */
int hsumma_model_cost(int32_t algo, const hsumma_platform* pf, int64_t n, int32_t P, int32_t Q,
                      int32_t G, int64_t b, int64_t B, hsumma_cost* out);
/* Eq. (10): derivative in G of the Van de Geijn cost (square grid of p
 * processes, b = B); zero at G = sqrt(p), and G = sqrt(p) is the minimum in
 * (1, p) iff alpha / beta > 2 n b / p (eq. (11)). */
int hsumma_model_dcomm_dgroups(const hsumma_platform* pf, int64_t n, double p, double G,
                               int64_t b, double* derivative);
/* More than two levels of groups (the paper's future work, Sec. VI): level
 * l (0 = outermost, nlevels <= 16) arranges its units I[l] x J[l] (the
 * products over the levels must be P and Q) and moves blocks of width
 * blocks[l] (non-increasing): every such step broadcasts A's n blocks[l] / P
 * elements per process along J[l] units of a row and B's n blocks[l] / Q
 * along I[l] units of a column.  One level (P, Q) with b is SUMMA; two
 * levels (I, J), (P/I, Q/J) with (B, b) give hsumma_model_cost.  In `out`
 * the innermost level fills the *_inner terms and all other levels the
 * *_outer terms; per_level (nullable, nlevels entries) receives each
 * level's seconds. */
int hsumma_model_cost_levels(int32_t algo, const hsumma_platform* pf, int64_t n, int32_t P,
                             int32_t Q, int32_t nlevels, const int32_t* I, const int32_t* J,
                             const int64_t* blocks, hsumma_cost* out, double* per_level);
/* The G with the least modelled communication time over every group count
 * that the P x Q grid can arrange (costs within a relative 1e-12 of the
 * least go to the smaller G), its cost, and the cost of SUMMA (G = 1).  Any
 * output pointer may be null. */
int hsumma_model_select_groups(int32_t algo, const hsumma_platform* pf, int64_t n, int32_t P,
                               int32_t Q, int64_t b, int64_t B, int32_t* G_best,
                               hsumma_cost* best, hsumma_cost* summa);

/*
 * Learned cost model (the tuner's learned form): a 3-layer FP32 MLP
 *   Z = relu(relu(X W1 + b1) W2 + b2) W3 + b3
 * with X: N x F features per problem shape, H hidden units, and one output
 * per candidate kernel configuration (its predicted log run time).  All
 * pointers are device memory, row-major; `params` packs W1 (F x H), b1 (H),
 * W2 (H x H), b2 (H), W3 (H x K), b3 (K); `grads` has the same layout.
 * `work` holds hsumma_mlp_work_floats(N, H, K) floats.  Asynchronous on
 * `stream`.  Not part of the paper: it predicts the fastest configuration
 * so that exhaustive tuning can be skipped.
 */
int64_t hsumma_mlp_param_count(int32_t F, int32_t H, int32_t K);   /* -1 on bad dims */
int64_t hsumma_mlp_work_floats(int32_t N, int32_t H, int32_t K);
/* Z (N x K) = network(X) */
int hsumma_mlp_forward(int32_t N, int32_t F, int32_t H, int32_t K, const float* X,
                       const float* params, float* Z, float* work, void* stream);
/* Forward, masked mean squared error against T (mask 1 = timed candidate),
 * and gradients of that loss w.r.t. every parameter; *loss on device. */
int hsumma_mlp_grad(int32_t N, int32_t F, int32_t H, int32_t K, const float* X, const float* T,
                    const float* mask, const float* params, float* grads, float* Z, float* loss,
                    float* work, void* stream);
/* One Adam step (bias-corrected, step counts from 1) over n parameters. */
int hsumma_mlp_adam(int64_t n, float* params, const float* grads, float* m, float* v, float lr,
                    float beta1, float beta2, float eps, int32_t step, void* stream);

/* Message for the last failure on this thread ("" if none). */
const char* hsumma_last_error(void);

/* Library version string. */
const char* hsumma_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HSUMMA_H */
