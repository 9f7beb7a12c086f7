// LU factorisation without pivoting whose trailing-matrix update is the
// HSUMMA local update -- the second workload the paper names for its
// hierarchical panel updates (Sec. VI).
//
// A = L U in place (L unit lower, strictly below the diagonal; U upper), by
// blocked elimination with the two block sizes of Sec. III: outer panels of
// M columns, each factored in inner blocks of b columns.  For outer panel
// [J, J + w) and each inner block [j, j + v) of it:
//   1. factor the v x v diagonal block (textbook elimination) and solve
//      L21 = A21 U11^-1 for every row below it; -L21 is also written to the
//      workspace, so the updates below are C += A B;
//   2. U12 = L11^-1 A12 for every column right of the block;
//   3. the update inside the outer panel, A[j+v:, j+v:J+w] -= L21 U12, and
//      on the outer panel's own rows right of it, A[j+v:J+w, J+w:] -= L U12
//      (one dense FP64 launch over the L-shaped block, k = v).
// Then the trailing matrix A[J+w:, J+w:] -= L21 U12 with k = w is one
// HSUMMA outer update on the P x Q grid with G groups (any precision form):
// C is loaded once, held in MFMA accumulators across the w/b inner steps
// and stored once -- the outer block's role on one GPU.
//
// No pivoting: the caller guarantees nonzero leading principal minors (e.g.
// a diagonally dominant matrix); a zero pivot gives Inf or NaN factors.
#include <algorithm>
#include <cstring>
#include <new>
#include <type_traits>
#include <vector>

#include "internal.h"

namespace hs {

constexpr int kLuMaxB = 64;          // inner block: the diagonal block lives in LDS
constexpr int kLuThreads = 256;

// Factor the v x v diagonal block at (j, j) in LDS, then for the rows
// j + v + 256 * blockIdx.x + thread: L21 row = A21 row U11^-1 (forward
// substitution in the order of textbook elimination), written in place and
// negated into negL (row r at negL + (r - J) * ldl + (j - J)).  Workgroup 0
// also writes the factored block back.
__global__ __launch_bounds__(kLuThreads) void lu_panel_kernel(double* A, int64_t lda, int n,
                                                               int j, int v, double* negL,
                                                               int64_t ldl, int J) {
  __shared__ double D[kLuMaxB][kLuMaxB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < v * v; e += kLuThreads)
    D[e / v][e % v] = A[(int64_t)(j + e / v) * lda + j + e % v];
  __syncthreads();
  for (int c = 0; c < v; ++c) {
    const double piv = D[c][c];
    for (int r = c + 1 + tid; r < v; r += kLuThreads) D[r][c] = D[r][c] / piv;
    __syncthreads();
    const int w2 = v - c - 1;
    for (int e = tid; e < w2 * w2; e += kLuThreads) {
      const int r = c + 1 + e / w2, cc = c + 1 + e % w2;
      D[r][cc] = D[r][cc] - D[r][c] * D[c][cc];
    }
    __syncthreads();
  }
  if (blockIdx.x == 0)
    for (int e = tid; e < v * v; e += kLuThreads)
      A[(int64_t)(j + e / v) * lda + j + e % v] = D[e / v][e % v];
  const int r = j + v + (int)blockIdx.x * kLuThreads + tid;
  if (r >= n) return;
  double x[kLuMaxB];
  double* row = A + (int64_t)r * lda + j;
#pragma unroll
  for (int c = 0; c < kLuMaxB; ++c) x[c] = c < v ? row[c] : 0.0;
#pragma unroll
  for (int k = 0; k < kLuMaxB; ++k) {
    if (k < v) {
      x[k] = x[k] / D[k][k];
#pragma unroll
      for (int c = k + 1; c < kLuMaxB; ++c)
        if (c < v) x[c] = x[c] - x[k] * D[k][c];
    }
  }
  double* nl = negL + (int64_t)(r - J) * ldl + (j - J);
#pragma unroll
  for (int c = 0; c < kLuMaxB; ++c)
    if (c < v) {
      row[c] = x[c];
      nl[c] = -x[c];
    }
}

// U12 = L11^-1 A12 for the columns [c0, c1) right of the factored v x v
// block at (j, j): one column per thread (unit lower forward substitution,
// in the order of textbook elimination), in place.
__global__ __launch_bounds__(kLuThreads) void lu_row_solve_kernel(double* A, int64_t lda, int j,
                                                                   int v, int c0, int c1) {
  __shared__ double Lw[kLuMaxB][kLuMaxB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < v * v; e += kLuThreads)
    Lw[e / v][e % v] = A[(int64_t)(j + e / v) * lda + j + e % v];
  __syncthreads();
  const int col = c0 + (int)blockIdx.x * kLuThreads + tid;
  if (col >= c1) return;
  double y[kLuMaxB];
#pragma unroll
  for (int r = 0; r < kLuMaxB; ++r) y[r] = r < v ? A[(int64_t)(j + r) * lda + col] : 0.0;
#pragma unroll
  for (int k = 0; k < kLuMaxB; ++k) {
    if (k < v) {
#pragma unroll
      for (int r = k + 1; r < kLuMaxB; ++r)
        if (r < v) y[r] = y[r] - Lw[r][k] * y[k];
    }
  }
#pragma unroll
  for (int r = 0; r < kLuMaxB; ++r)
    if (r < v) A[(int64_t)(j + r) * lda + col] = y[r];
}

// ---- full blocks of a compile-time width V (no per-element guards) ---------
// One wave factors the V x V diagonal block: lane t holds row t; at step c
// lane c publishes its (final) row through LDS and every lane below it
// eliminates with it.  The block is written back in place.
template <int V>
__global__ __launch_bounds__(64) void lu_diag_kernel(double* A, int64_t lda, int j) {
  __shared__ double prow[V];
  const int t = threadIdx.x;
  double x[V];
  double* row = A + (int64_t)(j + min(t, V - 1)) * lda + j;
#pragma unroll
  for (int c = 0; c < V; ++c) x[c] = row[c];
#pragma unroll
  for (int c = 0; c < V; ++c) {
    if (t == c) {
#pragma unroll
      for (int cc = c; cc < V; ++cc) prow[cc] = x[cc];
    }
    __syncthreads();
    if (t > c && t < V) {
      x[c] = x[c] / prow[c];
#pragma unroll
      for (int cc = c + 1; cc < V; ++cc) x[cc] = x[cc] - x[c] * prow[cc];
    }
    __syncthreads();
  }
  if (t < V) {
#pragma unroll
    for (int c = 0; c < V; ++c) row[c] = x[c];
  }
}

// The two triangular solves that depend only on the factored diagonal block,
// in one launch (straight-line code: every step works on the shrinking
// triangle only).  Workgroups [0, nrow): L21 = A21 U11^-1 for the rows
// j + V + 64 * blockIdx.x + lane (U11 from LDS), in place and negated into
// negL.  The rest: U12 = L11^-1 A12 for the columns c0 + 64 * (blockIdx.x -
// nrow) + lane, with L11 kept transposed in LDS so that the multipliers of
// one step are contiguous.
template <int V>
__global__ __launch_bounds__(64) void lu_solve_kernel(double* A, int64_t lda, int n, int j,
                                                       int nrow, int c0, double* negL,
                                                       int64_t ldl, int J) {
  __shared__ double T[V][V + 1];
  const int t = threadIdx.x;
  const bool rows = (int)blockIdx.x < nrow;
  const double* D = A + (int64_t)j * lda + j;
  for (int e = t; e < V * V; e += 64) {
    const double d = D[(int64_t)(e / V) * lda + e % V];
    if (rows) T[e / V][e % V] = d;
    else T[e % V][e / V] = d;
  }
  __syncthreads();
  double x[V];
  if (rows) {
    const int r = j + V + (int)blockIdx.x * 64 + t;
    if (r >= n) return;
    double* row = A + (int64_t)r * lda + j;
#pragma unroll
    for (int c = 0; c < V; ++c) x[c] = row[c];
#pragma unroll
    for (int k = 0; k < V; ++k) {
      x[k] = x[k] / T[k][k];
#pragma unroll
      for (int c = k + 1; c < V; ++c) x[c] = x[c] - x[k] * T[k][c];
    }
    double* nl = negL + (int64_t)(r - J) * ldl + (j - J);
#pragma unroll
    for (int c = 0; c < V; ++c) {
      row[c] = x[c];
      nl[c] = -x[c];
    }
    return;
  }
  const int col = c0 + ((int)blockIdx.x - nrow) * 64 + t;
  if (col >= n) return;
  double* cp = A + (int64_t)j * lda + col;
#pragma unroll
  for (int r = 0; r < V; ++r) x[r] = cp[(int64_t)r * lda];
#pragma unroll
  for (int k = 0; k < V; ++k)
#pragma unroll
    for (int r = k + 1; r < V; ++r) x[r] = x[r] - T[k][r] * x[k];
#pragma unroll
  for (int r = 0; r < V; ++r) cp[(int64_t)r * lda] = x[r];
}

// The panel steps of one inner block [j, j + v): the fast kernels when v is
// 16, 32 or 64, else the general ones above.
hipError_t lu_panel_step(double* A, int64_t lda, int n, int j, int v, double* negL, int64_t ldl,
                         int J, hipStream_t s) {
  const int below = n - j - v, right = n - j - v;
  auto fast = [&](auto vc) {
    constexpr int V = decltype(vc)::value;
    hipLaunchKernelGGL(lu_diag_kernel<V>, dim3(1), dim3(64), 0, s, A, lda, j);
    const int nrow = (below + 63) / 64, ncol = (right + 63) / 64;
    if (nrow + ncol > 0)
      hipLaunchKernelGGL(lu_solve_kernel<V>, dim3(nrow + ncol), dim3(64), 0, s, A, lda, n, j,
                         nrow, j + v, negL, ldl, J);
  };
  if (v == 64) fast(std::integral_constant<int, 64>{});
  else if (v == 32) fast(std::integral_constant<int, 32>{});
  else if (v == 16) fast(std::integral_constant<int, 16>{});
  else {
    const int wgs = std::max(1, (below + kLuThreads - 1) / kLuThreads);
    hipLaunchKernelGGL(lu_panel_kernel, dim3(wgs), dim3(kLuThreads), 0, s, A, lda, n, j, v, negL,
                       ldl, J);
    if (right > 0)
      hipLaunchKernelGGL(lu_row_solve_kernel, dim3((right + kLuThreads - 1) / kLuThreads),
                         dim3(kLuThreads), 0, s, A, lda, j, v, j + v, n);
  }
  return hipGetLastError();
}

}  // namespace hs

using hs::set_error;

namespace {

struct LuOuter {
  int64_t J, w;
  int64_t w2 = 0;                     // width of the next outer panel (0: last panel)
  // without look-ahead: C = A[J+w:, J+w:], k = w (null when empty)
  hsumma_plan_t trailing = nullptr;
  // with look-ahead, the same update in three parts: the next panel's rows
  // and columns first, the rest concurrently with that panel's factorisation
  hsumma_plan_t cross_rows = nullptr;   // C = A[J+w:J+w+w2, J+w:]
  hsumma_plan_t cross_cols = nullptr;   // C = A[J+w+w2:, J+w:J+w+w2]
  hsumma_plan_t rest = nullptr;         // C = A[J+w+w2:, J+w+w2:]
};

int lu_invalid(const std::string& msg) {
  set_error(msg);
  return HSUMMA_ERR_INVALID;
}

}  // namespace

struct hsumma_lu_plan_s {
  int64_t n = 0, b = 0, M = 0;
  bool lookahead = false;
  std::vector<LuOuter> outer;
  size_t off_negL = 0, negL_bytes = 0, off_sub = 0, off_aux = 0, sub_bytes = 0, aux_bytes = 0,
         ws_bytes = 0;
  // look-ahead: a second stream and two events, made on first use on a device
  int device = -1;
  hipStream_t aux = nullptr;
  hipEvent_t panel_done = nullptr, rest_done = nullptr;
  ~hsumma_lu_plan_s() {
    for (auto& o : outer)
      for (hsumma_plan_t q : {o.trailing, o.cross_rows, o.cross_cols, o.rest})
        if (q) hsumma_plan_destroy(q);
    if (aux) {
      int cur = -1;
      if (hipGetDevice(&cur) != hipSuccess) cur = -1;
      if (device >= 0 && device != cur) (void)hipSetDevice(device);
      (void)hipEventDestroy(panel_done);
      (void)hipEventDestroy(rest_done);
      (void)hipStreamDestroy(aux);
      if (cur >= 0 && device != cur) (void)hipSetDevice(cur);
    }
  }
};

namespace {

// An HSUMMA plan for C (rows x cols) += A (rows x k) B (k x cols) on the
// P x Q grid (clamped to the block) with G groups where they can be arranged;
// *need grows to its workspace size.
int update_plan(int64_t rows, int64_t cols, int64_t k, int32_t P, int32_t Q, int32_t G,
                int64_t b, const hsumma_opts& o, bool concurrent, hsumma_plan_t* out,
                size_t* need) {
  hsumma_opts t = o;
  t.m = rows;
  t.k = k;
  t.lookahead = 0;
  // FP64: 128 x 128 macro-tiles (64 x 64 below 512 rows or columns) unless
  // the caller names a tile.  The plan's own rule looks at the processor
  // tile, which the thin block-row and block-column updates of the
  // look-ahead make small; its 64 x 64 choice there made the look-ahead 7 %
  // slower at n = 16384, M = 2048, and its 128 x 64 choice for M >= 1024 is
  // slower at one workgroup per CU.
  if (t.prec == HSUMMA_FP64 && !t.tile_m && !t.tile_n && !t.kc) {
    t.tile_m = t.tile_n = (rows < 512 || cols < 512) ? 64 : 128;
    t.kc = 16;
  }
  if (concurrent) {
    // runs beside the panel kernels: a persistent launch that leaves room
    // on every CU (one workgroup per CU unless the caller says otherwise)
    t.persistent = 1;
    if (!t.wgs_per_cu) t.wgs_per_cu = 1;
  }
  const int32_t tp = (int32_t)std::min<int64_t>(P, rows), tq = (int32_t)std::min<int64_t>(Q, cols);
  int I = 0, Jg = 0;
  const int32_t tg = hs::factor_groups(tp, tq, G, &I, &Jg) ? G : 1;
  const int64_t tb = std::min(b, k);
  const int64_t tM = (k + tb - 1) / tb * tb;
  int rc = hsumma_plan(out, cols, tp, tq, tg, tb, tM, &t);
  if (rc) return rc;
  size_t bytes = 0;
  hsumma_workspace_size(*out, &bytes);
  *need = std::max(*need, bytes);
  return HSUMMA_OK;
}

}  // namespace

extern "C" {

int hsumma_lu_plan(hsumma_lu_plan_t* out, int64_t n, int32_t P, int32_t Q, int32_t G, int64_t b,
                   int64_t M, const hsumma_opts* opts) {
  if (!out) return lu_invalid("null output pointer");
  *out = nullptr;
  if (n < 1 || n >= (int64_t(1) << 31)) return lu_invalid("n must be in [1, 2^31)");
  if (b < 1 || b > hs::kLuMaxB) return lu_invalid("inner block b must be in [1, 64]");
  if (M < b || M % b) return lu_invalid("outer block M must be a positive multiple of b");
  if (P < 1 || Q < 1 || G < 1) return lu_invalid("P, Q and G must be >= 1");
  hsumma_opts o;
  hsumma_opts_default(&o);
  if (opts) o = *opts;
  if (o.m || o.k) return lu_invalid("the LU factorisation is square: leave opts.m and opts.k 0");
  hsumma_lu_plan_s* p = new (std::nothrow) hsumma_lu_plan_s();
  if (!p) return lu_invalid("out of host memory");
  p->n = n; p->b = b; p->M = M;
  p->lookahead = o.lookahead != 0;
  size_t sub = 256, aux = 256;
  for (int64_t J = 0; J < n; J += M) {
    LuOuter lo;
    lo.J = J;
    lo.w = std::min(M, n - J);
    const int64_t tail = n - J - lo.w;
    int rc = HSUMMA_OK;
    if (tail > 0 && !p->lookahead) {
      rc = update_plan(tail, tail, lo.w, P, Q, G, b, o, false, &lo.trailing, &sub);
    } else if (tail > 0) {
      lo.w2 = std::min(M, tail);
      const int64_t rest = tail - lo.w2;
      rc = update_plan(lo.w2, tail, lo.w, P, Q, G, b, o, false, &lo.cross_rows, &sub);
      if (!rc && rest > 0)
        rc = update_plan(rest, lo.w2, lo.w, P, Q, G, b, o, false, &lo.cross_cols, &sub);
      if (!rc && rest > 0)
        rc = update_plan(rest, rest, lo.w, P, Q, G, b, o, true, &lo.rest, &aux);
    }
    p->outer.push_back(lo);
    if (rc) {
      delete p;
      return rc;
    }
  }
  // 4 KiB units: the trailing updates' own workspaces (digit planes of the
  // split forms) then start on 4 KiB boundaries of a 4 KiB-aligned workspace
  auto al = [](size_t x) { return (x + 4095) & ~(size_t)4095; };
  // the negated L21 panel: two buffers with look-ahead (the next panel is
  // written while the rest of the trailing update still reads this one)
  p->negL_bytes = al((size_t)n * (size_t)M * sizeof(double));
  p->off_negL = 0;
  p->off_sub = p->negL_bytes * (p->lookahead ? 2 : 1);
  p->sub_bytes = al(sub);
  p->off_aux = p->off_sub + p->sub_bytes;
  p->aux_bytes = p->lookahead ? al(aux) : 0;
  p->ws_bytes = p->off_aux + p->aux_bytes;
  *out = p;
  return HSUMMA_OK;
}

void hsumma_lu_plan_destroy(hsumma_lu_plan_t p) { delete p; }

int hsumma_lu_workspace_size(hsumma_lu_plan_t p, size_t* bytes) {
  if (!p || !bytes) return lu_invalid("null argument");
  *bytes = p->ws_bytes;
  return HSUMMA_OK;
}

int hsumma_lu(hsumma_lu_plan_t p, double* A, int64_t lda, void* ws, size_t ws_bytes,
              void* stream) {
  if (!p) return lu_invalid("null plan");
  if (!A || (((uintptr_t)A) & 7)) return lu_invalid("A must be a non-null 8-byte-aligned pointer");
  if (lda < p->n) return lu_invalid("lda smaller than n");
  if (!ws || ws_bytes < p->ws_bytes) {
    set_error("workspace missing or smaller than hsumma_lu_workspace_size()");
    return HSUMMA_ERR_WORKSPACE;
  }
  if (((uintptr_t)ws) & 255) return lu_invalid("workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  auto check = [&](hipError_t e, const char* what) {
    if (e == hipSuccess) return HSUMMA_OK;
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return HSUMMA_ERR_DEVICE;
  };
  if (p->lookahead) {
    int dev = 0;
    int rc = check(hipGetDevice(&dev), "hipGetDevice");
    if (rc) return rc;
    if (p->aux && p->device != dev) {
      set_error("an LU plan with look-ahead is used on one device only");
      return HSUMMA_ERR_INVALID;
    }
    if (!p->aux) {
      if ((rc = check(hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking), "aux stream")))
        return rc;
      if ((rc = check(hipEventCreateWithFlags(&p->panel_done, hipEventDisableTiming), "event")))
        return rc;
      if ((rc = check(hipEventCreateWithFlags(&p->rest_done, hipEventDisableTiming), "event")))
        return rc;
      p->device = dev;
    }
  }
  const int64_t n = p->n, M = p->M;
  uint8_t* w8 = (uint8_t*)ws;
  void* sub = w8 + p->off_sub;
  void* auxws = w8 + p->off_aux;
  bool rest_pending = false;
  for (size_t oi = 0; oi < p->outer.size(); ++oi) {
    const LuOuter& o = p->outer[oi];
    const int64_t J = o.J, w = o.w;
    double* negL = (double*)(w8 + p->off_negL + (p->lookahead ? (oi & 1) * p->negL_bytes : 0));
    for (int64_t j = J; j < J + w; j += p->b) {
      const int64_t v = std::min(p->b, J + w - j);
      const int64_t below = n - j - v;
      int rc = check(hs::lu_panel_step(A, lda, (int)n, (int)j, (int)v, negL, M, (int)J, s),
                     "LU panel launch");
      if (rc) return rc;
      // in one launch: inside the outer panel, A[j+v:n, j+v:J+w] += (-L21)
      // U12, and the outer panel's rows right of it, A[j+v:J+w, J+w:n] +=
      // (-L) U12 (the same -L rows and U12 row block, an L-shaped C)
      const double* nl = negL + (j + v - J) * M + (j - J);
      const int64_t inside = J + w - j - v;
      if (inside > 0) {
        rc = check(hs::launch_fp64_dense(nl, M, A + j * lda + (j + v), lda,
                                         A + (j + v) * lda + (j + v), lda, below, inside, v, s,
                                         inside, n - J - w),
                   "LU panel update launch");
        if (rc) return rc;
      }
    }
    const double* L21 = negL + w * M;          // rows J + w .. n of -L21
    const double* U12 = A + J * lda + (J + w);  // rows J .. J + w of U, right of the panel
    if (!p->lookahead) {
      if (o.trailing) {
        int rc = hsumma_outer_update(o.trailing, 0, L21, M, U12, lda, A + (J + w) * lda + (J + w),
                                     lda, sub, p->sub_bytes, stream);
        if (rc) return rc;
      }
      continue;
    }
    if (!o.cross_rows) continue;
    // the previous panel's rest of the trailing update covers this one's
    // trailing block: it must be done before any part of the new update
    if (rest_pending) {
      int rc = check(hipStreamWaitEvent(s, p->rest_done, 0), "wait for the trailing update");
      if (rc) return rc;
      rest_pending = false;
    }
    const int64_t w2 = o.w2;
    if (o.rest) {
      // the rest on the second stream, once this panel's factors are ready
      int rc = check(hipEventRecord(p->panel_done, s), "record panel");
      if (!rc) rc = check(hipStreamWaitEvent(p->aux, p->panel_done, 0), "wait panel");
      if (!rc) rc = hsumma_outer_update(o.rest, 0, L21 + w2 * M, M, U12 + w2, lda,
                                        A + (J + w + w2) * lda + (J + w + w2), lda, auxws,
                                        p->aux_bytes, (void*)p->aux);
      if (!rc) rc = check(hipEventRecord(p->rest_done, p->aux), "record rest");
      if (rc) return rc;
      rest_pending = true;
    }
    // the next panel's rows and columns on this stream, then its factorisation
    int rc = hsumma_outer_update(o.cross_rows, 0, L21, M, U12, lda, A + (J + w) * lda + (J + w),
                                 lda, sub, p->sub_bytes, stream);
    if (!rc && o.cross_cols)
      rc = hsumma_outer_update(o.cross_cols, 0, L21 + w2 * M, M, U12, lda,
                               A + (J + w + w2) * lda + (J + w), lda, sub, p->sub_bytes, stream);
    if (rc) return rc;
  }
  if (rest_pending) {
    int rc = check(hipStreamWaitEvent(s, p->rest_done, 0), "wait for the trailing update");
    if (rc) return rc;
  }
  return HSUMMA_OK;
}

}  // extern "C"
