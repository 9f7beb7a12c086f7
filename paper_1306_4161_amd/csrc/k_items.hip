// Work-item table of a plan, generated on the device into the caller's
// workspace (so the library neither allocates device memory nor copies host
// data to the device).
//
// A work item is one macro-tile of one virtual processor's C tile (Sec. II-A:
// processor (i, j) owns a block of C; Sec. III: processors are arranged in
// I x J groups).  The table lists the items group by group -- group (x, y),
// then processor (i, j) inside it, then the processor's macro-tiles in blocks
// of br x bc -- and is cut into 8 contiguous lists, one per XCD.  For the
// persistent launch mode and the split forms each list is then put in
// longest-first order (stable by area), so that the static round-robin of a
// persistent grid stays balanced on uneven tiles.  The host builds the same
// table (the plan's definition of the order); the two are compared bit for
// bit by the tests.
//
// One workgroup of 1024 threads per XCD list, independent of the others:
// (1) item counts of every processor and their prefix sums, in LDS; (2) the
// list's items, one per thread-iteration (the processor by binary search
// over the prefix sums, then closed-form piece coordinates); (3) in the
// longest-first modes, a stable partition of the list by area in decreasing
// order (one pass per distinct area).
#include "internal.h"

namespace hs {

namespace {

constexpr int kGenThreads = 1024;

// Pieces (macro-tile rows or columns of width t) of processor r along a
// dimension of length len split into `parts` processors.
__device__ int32_t gen_npieces(const ItemGenArgs& g, bool rows, int r) {
  const int64_t len = rows ? g.m : g.n;
  const int parts = rows ? g.P : g.Q;
  const int t = rows ? g.tm : g.tn;
  if (g.dist == HSUMMA_DIST_BLOCK) {
    const int64_t lo = (int64_t)r * len / parts, hi = (int64_t)(r + 1) * len / parts;
    return (int32_t)((hi - lo + t - 1) / t);
  }
  const int32_t nb = (int32_t)g.nb;
  const int32_t nblk = (int32_t)((len + nb - 1) / nb);
  if (r >= nblk) return 0;
  const int32_t runs = (nblk - 1 - r) / parts + 1;          // blocks r, r + parts, ...
  const int32_t ppr = (nb + t - 1) / t;                     // pieces of a full block
  const int32_t last = r + (runs - 1) * parts;
  const int32_t tail = (int32_t)(len - (int64_t)last * nb);  // length of the last block
  if (last == nblk - 1 && tail < nb) return (runs - 1) * ppr + (tail + t - 1) / t;
  return runs * ppr;
}

// Global [g0, g1) of piece idx of processor r.
__device__ void gen_piece(const ItemGenArgs& g, bool rows, int r, int32_t idx, int32_t* g0,
                          int32_t* g1) {
  const int64_t len = rows ? g.m : g.n;
  const int parts = rows ? g.P : g.Q;
  const int t = rows ? g.tm : g.tn;
  if (g.dist == HSUMMA_DIST_BLOCK) {
    const int32_t lo = (int32_t)((int64_t)r * len / parts);
    const int32_t hi = (int32_t)((int64_t)(r + 1) * len / parts);
    *g0 = lo + idx * t;
    *g1 = (int32_t)min((int64_t)*g0 + t, (int64_t)hi);
    return;
  }
  const int32_t nb = (int32_t)g.nb;
  const int32_t ppr = (nb + t - 1) / t;
  const int32_t run = idx / ppr, within = idx - run * ppr;
  const int64_t blk = r + (int64_t)run * parts;
  *g0 = (int32_t)(blk * nb) + within * t;
  *g1 = (int32_t)min((int64_t)*g0 + t, min((blk + 1) * nb, len));
}

// Processor of rank r in group order: groups (x, y) row-major, processors
// (i, j) row-major inside a group.
__device__ void gen_proc(const ItemGenArgs& g, int r, int* pr, int* pc) {
  const int gp = g.P / g.I, gq = g.Q / g.J;
  const int j = r % gq;
  r /= gq;
  const int i = r % gp;
  r /= gp;
  const int y = r % g.J, x = r / g.J;
  *pr = x * gp + i;
  *pc = y * gq + j;
}

__device__ int32_t gen_count(const ItemGenArgs& g, int r) {
  int pr, pc;
  gen_proc(g, r, &pr, &pc);
  return gen_npieces(g, true, pr) * gen_npieces(g, false, pc);
}

// Exclusive scan of one value per thread over the workgroup; *total gets the
// sum.  Ends with a barrier, so `buf` may be reused at once.
__device__ int64_t block_exclusive_scan(int64_t v, int64_t* buf, int64_t* total) {
  const int tid = threadIdx.x;
  buf[tid] = v;
  __syncthreads();
  for (int off = 1; off < kGenThreads; off <<= 1) {
    const int64_t add = tid >= off ? buf[tid - off] : 0;
    __syncthreads();
    buf[tid] += add;
    __syncthreads();
  }
  const int64_t incl = buf[tid];
  *total = buf[kGenThreads - 1];
  __syncthreads();
  return incl - v;
}

__device__ int64_t block_max(int64_t v, int64_t* buf) {
  const int tid = threadIdx.x;
  buf[tid] = v;
  __syncthreads();
  for (int off = kGenThreads / 2; off > 0; off >>= 1) {
    if (tid < off) buf[tid] = max(buf[tid], buf[tid + off]);
    __syncthreads();
  }
  const int64_t r = buf[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ int64_t area(const WorkItem& w) { return (int64_t)w.h * w.w; }

}  // namespace

__global__ __launch_bounds__(kGenThreads) void gen_items_kernel(ItemGenArgs g) {
  __shared__ int64_t buf[kGenThreads];
  __shared__ int32_t prefix[kGenMaxProcs + 1];
  const int tid = threadIdx.x;
  const int nproc = g.P * g.Q;                 // <= kGenMaxProcs (checked by the plan)
  const int x = blockIdx.x;                    // this workgroup's XCD list

  // (1) per-processor item counts, exclusive prefix sums in group order
  const int chunk = (nproc + kGenThreads - 1) / kGenThreads;
  const int r0 = min(nproc, tid * chunk), r1 = min(nproc, r0 + chunk);
  int64_t local = 0;
  for (int r = r0; r < r1; ++r) local += gen_count(g, r);
  int64_t total = 0;
  int64_t run = block_exclusive_scan(local, buf, &total);
  for (int r = r0; r < r1; ++r) {
    prefix[r] = (int32_t)run;
    run += gen_count(g, r);
  }
  if (tid == 0) prefix[nproc] = (int32_t)total;
  __syncthreads();
  const int b0 = min(g.nitems, x * g.per_xcd), b1 = min(g.nitems, (x + 1) * g.per_xcd);
  if (total != g.nitems) {
    // the counts disagree with the plan's (never expected): a table of 1 x 1
    // items at the origin keeps every later access in bounds, and the test
    // that compares this table with the host's fails
    for (int u = b0 + tid; u < b1; u += kGenThreads) g.items[u] = WorkItem{0, 0, 1, 1};
    return;
  }

  // (2) this list's items in group order
  WorkItem* out = g.lpt ? g.tmp : g.items;
  for (int u = b0 + tid; u < b1; u += kGenThreads) {
    int lo = 0, hi = nproc - 1;                 // largest r with prefix[r] <= u
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (prefix[mid] <= u) lo = mid;
      else hi = mid - 1;
    }
    const int r = lo;
    int pr, pc;
    gen_proc(g, r, &pr, &pc);
    const int32_t nr = gen_npieces(g, true, pr), nc = gen_npieces(g, false, pc);
    const int32_t t = u - prefix[r];
    // blocks of br x bc pieces, row-major; pieces row-major inside a block
    const int32_t row_block = g.br * nc;
    const int32_t tb = t / row_block, rb = tb * g.br;
    const int32_t rows_in = min(g.br, nr - rb);
    const int32_t t2 = t - tb * row_block;
    const int32_t col_block = rows_in * g.bc;
    const int32_t tc = t2 / col_block, cb = tc * g.bc;
    const int32_t cols_in = min(g.bc, nc - cb);
    const int32_t t3 = t2 - tc * col_block;
    const int32_t ri = t3 / cols_in;
    int32_t a0, a1, c0, c1;
    gen_piece(g, true, pr, rb + ri, &a0, &a1);
    gen_piece(g, false, pc, cb + (t3 - ri * cols_in), &c0, &c1);
    out[u] = WorkItem{a0, c0, a1 - a0, c1 - c0};
  }
  if (!g.lpt) return;
  __threadfence_block();
  __syncthreads();

  // (3) the list in longest-first order, stable: one pass per distinct area,
  // largest first, each a stable compaction of that area's items
  const int L = b1 - b0;
  if (L <= 0) return;                          // uniform over the workgroup
  const int ch = (L + kGenThreads - 1) / kGenThreads;
  const int i0 = b0 + min(L, tid * ch), i1 = b0 + min(L, tid * ch + ch);
  int64_t below = INT64_MAX;                   // areas placed so far are >= below
  int64_t placed = 0;
  while (placed < L) {
    int64_t mk = -1;
    for (int i = i0; i < i1; ++i) {
      const int64_t a = area(g.tmp[i]);
      if (a < below) mk = max(mk, a);
    }
    mk = block_max(mk, buf);
    if (mk < 0) break;                         // nothing left (uniform)
    int64_t cnt = 0;
    for (int i = i0; i < i1; ++i) cnt += area(g.tmp[i]) == mk;
    int64_t n_mk = 0;
    int64_t pos = b0 + placed + block_exclusive_scan(cnt, buf, &n_mk);
    for (int i = i0; i < i1; ++i)
      if (area(g.tmp[i]) == mk) g.items[pos++] = g.tmp[i];
    placed += n_mk;
    below = mk;
  }
}

hipError_t launch_gen_items(const ItemGenArgs& g, hipStream_t s) {
  if (g.nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(gen_items_kernel, dim3(8), dim3(kGenThreads), 0, s, g);
  return hipGetLastError();
}

}  // namespace hs
