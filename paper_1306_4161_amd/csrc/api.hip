// C ABI of the Hierarchical SUMMA local-update library: plans, the step
// schedule, work-item tables and the launch sequence.
//
// Plan (Sec. III, Alg. 1): the P x Q grid is arranged as I x J groups; the
// k dimension is consumed in outer blocks of M and inner blocks of b.  Each
// virtual processor's C tile is cut into macro-tiles (work items).  The
// items are ordered group by group and tile by tile, and that list is cut
// into 8 contiguous parts, one per XCD: the processors of a group share an
// L2, the GPU's image of the paper's group-level broadcast.
//
// Device memory: the library allocates none.  Every compute call writes the
// plan's work-item table into the caller's workspace with one small kernel
// (k_items.hip) before its update launches, so a call depends on nothing but
// its arguments, and a captured graph regenerates the table on each replay.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "internal.h"
#include "split.h"

namespace hs {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

// Most square I x J = G with I | P, J | Q; ties to the smaller I.
bool factor_groups(int P, int Q, int G, int* I, int* J) {
  bool found = false;
  double best_ratio = 0;
  for (int i = 1; i <= P; ++i) {
    if (P % i || G % i) continue;
    int j = G / i;
    if (j > Q || Q % j) continue;
    double ratio = (double)std::max(i, j) / (double)std::min(i, j);
    if (!found || ratio < best_ratio) {
      found = true;
      best_ratio = ratio;
      *I = i;
      *J = j;
    }
  }
  return found;
}

}  // namespace hs

using hs::set_error;

namespace {

struct StepRec {
  int64_t k0, k1, outer;
};

struct GraphKey {
  const void* A; int64_t lda; const void* B; int64_t ldb; void* C; int64_t ldc;
  void* ws; void* stream;
  bool operator==(const GraphKey& o) const {
    return A == o.A && lda == o.lda && B == o.B && ldb == o.ldb && C == o.C &&
           ldc == o.ldc && ws == o.ws && stream == o.stream;
  }
};

}  // namespace

struct hsumma_plan_s {
  int64_t m = 0, n = 0, k = 0, b = 0, M = 0, nb = 0;
  int32_t P = 0, Q = 0, G = 0, I = 0, J = 0;
  hsumma_opts opts{};
  hs::TileCfg cfg{};
  std::vector<int64_t> rlo, clo, kqlo, kplo;  // block-distribution boundaries
  std::vector<StepRec> steps;
  std::vector<int64_t> outer_lo;              // k start of each outer step (+ end)
  std::vector<hs::WorkItem> items;
  int32_t per_xcd = 0;
  int32_t br = 1, bc = 1;      // macro-tiles per block inside a processor's tile
  bool lpt = false;            // XCD lists in longest-first order
  bool items_even = false;     // every work item starts at an even column, has even width
  // workspace layout (byte offsets): the work-item table (every precision),
  // then the precision form's digit planes, exponents and statistics
  size_t off_items = 0, off_items_tmp = 0;
  int32_t fmt = -1;            // -1: FP64 path; 0: BF16, 1: FP8-e4m3, 2: INT8 digits
  int32_t Wp = 0;              // padded panel width
  size_t off_digA = 0, off_digB = 0, off_eA = 0, off_fB = 0, off_part = 0, off_stats = 0,
         off_slices = 0, off_dump = 0, ws_bytes = 0;
  // split forms with look-ahead: a second set of digit planes, exponents and
  // partial statistics (panel g uses set g % 2), the second stream and its
  // events
  bool lookahead = false;
  size_t off_digA1 = 0, off_digB1 = 0, off_eA1 = 0, off_fB1 = 0, off_part1 = 0;
  hipStream_t aux = nullptr;
  hipEvent_t ev_start = nullptr, ev_split = nullptr, ev_prod = nullptr;
  int adevice = -1;
  std::mutex mu;
  bool have_graph = false;
  GraphKey gkey{};
  hipGraphExec_t gexec = nullptr;
  int gdevice = -1;
};

namespace {

#define HS_CHECK_HIP(expr)                                                         \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess) {                                                        \
      set_error(std::string(#expr) + ": " + hipGetErrorString(_e));                \
      return HSUMMA_ERR_DEVICE;                                                    \
    }                                                                              \
  } while (0)

int invalid(const std::string& msg) {
  set_error(msg);
  return HSUMMA_ERR_INVALID;
}

// Boundaries of a balanced block split of [0, len) into parts.
std::vector<int64_t> block_bounds(int64_t len, int parts) {
  std::vector<int64_t> lo(parts + 1);
  for (int r = 0; r <= parts; ++r) lo[r] = (int64_t)r * len / parts;
  return lo;
}

int owner_block(const std::vector<int64_t>& lo, int64_t g) {
  // largest r with lo[r] <= g
  auto it = std::upper_bound(lo.begin(), lo.end(), g);
  return (int)(it - lo.begin()) - 1;
}

// Global index runs owned by processor r along one dimension.
struct Run { int64_t g0, g1; };
std::vector<Run> runs_of(const hsumma_plan_s& p, bool rows, int r) {
  std::vector<Run> out;
  const int64_t len = rows ? p.m : p.n;
  const int parts = rows ? p.P : p.Q;
  if (p.opts.dist == HSUMMA_DIST_BLOCK) {
    const auto& lo = rows ? p.rlo : p.clo;
    if (lo[r + 1] > lo[r]) out.push_back({lo[r], lo[r + 1]});
  } else {
    for (int64_t blk = r; blk * p.nb < len; blk += parts)
      out.push_back({blk * p.nb, std::min((blk + 1) * p.nb, len)});
  }
  return out;
}

int64_t local_count(const hsumma_plan_s& p, bool rows, int r) {
  int64_t c = 0;
  for (auto& run : runs_of(p, rows, r)) c += run.g1 - run.g0;
  return c;
}

// Macro-tiles of width t over every processor's rows (or columns).
int64_t pieces_of(const hsumma_plan_s& p, bool rows, int64_t t) {
  int64_t c = 0;
  for (int r = 0; r < (rows ? p.P : p.Q); ++r)
    for (auto& run : runs_of(p, rows, r)) c += (run.g1 - run.g0 + t - 1) / t;
  return c;
}

// The FP64 macro-tile when the caller names none, from the number of
// macro-tiles a launch would have, the processors' tile size and the outer
// block.  A rule fitted to the tuner's exhaustive timings (2000 random
// shapes with m, n, k in [512, 16384], P, Q <= 16, M <= 512; twelve larger
// ones with M up to 1024; the 6 x 10 block-cyclic grid at n = 10000):
// within 2.5 % of the fastest candidate on average, where a fixed 128 x 128
// was 49 % behind on the random shapes.
//   * fewer than 768 items of 64 x 64: 32 x 32 (the launch needs the items);
//   * a processor tile under 512 on a side, an outer block under 128, or
//     fewer than 4096 items of 128 x 128: 64 x 64 (little work per item, or
//     128-wide tiles leave CUs idle or ragged);
//   * an outer block of 1024 or more: 128 x 64 (its two workgroups per CU
//     keep more C tiles in flight than 128 x 128 at the same reuse);
//   * otherwise 128 x 128.
hs::TileCfg default_tile(const hsumma_plan_s& p) {
  const int64_t i64 = pieces_of(p, true, 64) * pieces_of(p, false, 64);
  const int64_t i128 = pieces_of(p, true, 128) * pieces_of(p, false, 128);
  const int64_t side = std::min(p.m / p.P, p.n / p.Q);
  if (i64 < 768) return {32, 32, 16};
  if (side < 512 || p.M < 128 || i128 < 4096) return {64, 64, 16};
  if (p.M >= 1024) return {128, 64, 16};
  return {128, 128, 16};
}

// max_row_block: the largest br x (pieces of a processor column), the
// generator's int32 unit of a block row.
void build_items(hsumma_plan_s& p, int64_t* max_row_block) {
  const int gp = p.P / p.I, gq = p.Q / p.J;
  std::vector<std::vector<Run>> rpieces(p.P), cpieces(p.Q);
  for (int r = 0; r < p.P; ++r)
    for (auto& run : runs_of(p, true, r))
      for (int64_t g = run.g0; g < run.g1; g += p.cfg.tm)
        rpieces[r].push_back({g, std::min(g + p.cfg.tm, run.g1)});
  for (int c = 0; c < p.Q; ++c)
    for (auto& run : runs_of(p, false, c))
      for (int64_t g = run.g0; g < run.g1; g += p.cfg.tn)
        cpieces[c].push_back({g, std::min(g + p.cfg.tn, run.g1)});
  // Inside a tile the macro-tiles go in blocks of br x bc, sized so that the
  // workgroups one XCD runs at a time (32 CUs x occupancy) cover a square
  // of C: they then share the fewest A rows plus B columns per k-slice in
  // that XCD's L2.
  const int conc = 32 * (p.fmt < 0 ? std::max(1, hs::fp64_occupancy(p.cfg)) : 1);
  const int bc = std::max(1, (int)std::lround(std::sqrt((double)conc * p.cfg.tm / p.cfg.tn)));
  const int br = std::max(1, conc / bc);
  p.br = br;
  p.bc = bc;
  *max_row_block = 0;
  for (int c = 0; c < p.Q; ++c)
    *max_row_block = std::max<int64_t>(*max_row_block, (int64_t)br * cpieces[c].size());
  p.items.clear();
  for (int x = 0; x < p.I; ++x)
    for (int y = 0; y < p.J; ++y)
      for (int i = 0; i < gp; ++i)
        for (int j = 0; j < gq; ++j) {
          const int pr = x * gp + i, pc = y * gq + j;
          const size_t nr = rpieces[pr].size(), nc = cpieces[pc].size();
          for (size_t rb = 0; rb < nr; rb += br)
            for (size_t cb = 0; cb < nc; cb += bc)
              for (size_t ri = rb; ri < std::min(nr, rb + br); ++ri)
                for (size_t ci = cb; ci < std::min(nc, cb + bc); ++ci) {
                  const Run& rp = rpieces[pr][ri];
                  const Run& cp = cpieces[pc][ci];
                  p.items.push_back({(int32_t)rp.g0, (int32_t)cp.g0, (int32_t)(rp.g1 - rp.g0),
                                     (int32_t)(cp.g1 - cp.g0)});
                }
        }
  const int64_t nit = (int64_t)p.items.size();
  p.per_xcd = (int32_t)((nit + 7) / 8);
  p.items_even = true;
  for (auto& it : p.items)
    if ((it.c0 | it.w) & 1) p.items_even = false;
  p.lpt = p.opts.persistent || p.fmt >= 0;
  if (p.lpt) {
    // Longest-processing-time order inside each XCD's list, so that the
    // static round-robin of the persistent workgroups stays balanced when
    // tiles are uneven (ragged block-cyclic edges).
    for (int x = 0; x < 8; ++x) {
      auto b0 = p.items.begin() + std::min<int64_t>(nit, (int64_t)x * p.per_xcd);
      auto b1 = p.items.begin() + std::min<int64_t>(nit, (int64_t)(x + 1) * p.per_xcd);
      std::stable_sort(b0, b1, [](const hs::WorkItem& a, const hs::WorkItem& b) {
        return (int64_t)a.h * a.w > (int64_t)b.h * b.w;
      });
    }
  }
}

int check_ws(hsumma_plan_t p, const void* ws, size_t ws_bytes) {
  if (!ws || ws_bytes < p->ws_bytes) {
    set_error("workspace missing or smaller than hsumma_workspace_size()");
    return HSUMMA_ERR_WORKSPACE;
  }
  if (((uintptr_t)ws) & 255) return invalid("workspace must be 256-byte aligned");
  return HSUMMA_OK;
}

// Write the plan's work-item table into the workspace (one small kernel).
int prepare_items(hsumma_plan_t p, void* ws, hipStream_t stream) {
  if (p->items.empty()) return HSUMMA_OK;
  uint8_t* w8 = (uint8_t*)ws;
  hs::ItemGenArgs g;
  g.m = p->m; g.n = p->n;
  g.P = p->P; g.Q = p->Q; g.I = p->I; g.J = p->J;
  g.tm = p->cfg.tm; g.tn = p->cfg.tn; g.br = p->br; g.bc = p->bc;
  g.dist = p->opts.dist; g.nb = p->nb;
  g.nitems = (int32_t)p->items.size(); g.per_xcd = p->per_xcd; g.lpt = p->lpt ? 1 : 0;
  g.items = (hs::WorkItem*)(w8 + p->off_items);
  g.tmp = (hs::WorkItem*)(w8 + p->off_items_tmp);
  hipError_t e = hs::launch_gen_items(g, stream);
  if (e != hipSuccess) {
    set_error(std::string("work-item table launch: ") + hipGetErrorString(e));
    return HSUMMA_ERR_DEVICE;
  }
  return HSUMMA_OK;
}

int check_operands(hsumma_plan_t p, const double* A, int64_t lda, const double* B, int64_t ldb,
                   double* C, int64_t ldc) {
  if (!p) return invalid("null plan");
  if (!C || (p->k > 0 && (!A || !B))) return invalid("null matrix pointer");
  if (lda < std::max<int64_t>(1, p->k) || ldb < p->n || ldc < p->n)
    return invalid("leading dimension smaller than the row length");
  if (((uintptr_t)A | (uintptr_t)B | (uintptr_t)C) & 7)
    return invalid("matrix pointers must be 8-byte aligned");
  return HSUMMA_OK;
}

// Grid of a launch over the plan's items: one workgroup per item, or (the
// persistent mode, and always for the split forms) as many as the CUs hold.
int launch_grid(hsumma_plan_t p, bool persistent, int occ, int* grid) {
  *grid = 8 * p->per_xcd;
  if (persistent) {
    int dev = 0, cus = 0;
    HS_CHECK_HIP(hipGetDevice(&dev));
    HS_CHECK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (p->opts.wgs_per_cu > 0) occ = std::min(occ, (int)p->opts.wgs_per_cu);
    *grid = (int)std::min<int64_t>(*grid, (int64_t)cus * std::max(1, occ));
    *grid = std::max(8, (*grid / 8) * 8);
  }
  return HSUMMA_OK;
}

// The FP64 update over k-range [k0, k1) on every item of the table in the
// workspace, with the macro-tile `cfg`.  `gate`: see UpdateArgs.
int launch_fp64_range(hsumma_plan_t p, const hs::TileCfg& cfg, const double* A, int64_t lda,
                      const double* B, int64_t ldb, double* C, int64_t ldc, int64_t k0,
                      int64_t k1, int zero_init, bool persistent, const int32_t* gate, void* ws,
                      hipStream_t stream) {
  int grid = 0;
  int rc = launch_grid(p, persistent, hs::fp64_occupancy(cfg), &grid);
  if (rc) return rc;
  hs::UpdateArgs a{};
  a.A = A; a.lda = lda; a.B = B; a.ldb = ldb; a.C = C; a.ldc = ldc;
  a.items = (const hs::WorkItem*)((uint8_t*)ws + p->off_items);
  a.nitems = (int32_t)p->items.size(); a.per_xcd = p->per_xcd;
  a.k0 = k0; a.k1 = k1; a.bstep = p->b; a.zero_init = zero_init;
  a.persistent = persistent ? 1 : 0;
  a.gate = gate;
  // direct-to-LDS loads move 16-byte units: every k bound, leading
  // dimension and column offset must be even and the operands aligned;
  // the per-lane byte offsets (up to a tile's rows of A, 16 rows of B)
  // must stay below 2^31
  const bool dma = !p->opts.staged && hs::fp64_has_dma(cfg) && p->items_even &&
                   !((k0 | k1 | p->b | lda | ldb) & 1) &&
                   !(((uintptr_t)A | (uintptr_t)B) & 15) &&
                   (int64_t)cfg.tm * lda * 8 < (int64_t(1) << 31) &&
                   (int64_t)16 * ldb * 8 < (int64_t(1) << 31);
  hipError_t e = hs::launch_fp64(cfg, a, grid, stream, dma);
  if (e != hipSuccess) {
    set_error(std::string("fp64 update launch: ") + hipGetErrorString(e));
    return HSUMMA_ERR_DEVICE;
  }
  return HSUMMA_OK;
}

// The split of the panel k-range [k0, k1) of a precision form: its digit
// planes and exponents go to set `buf` of the workspace (set 1 exists with
// look-ahead only), its statistics and slice count to slot `slot`.
hs::SplitArgs split_args(hsumma_plan_t p, const double* A, int64_t lda, const double* B,
                         int64_t ldb, int64_t k0, int64_t k1, int64_t slot, int buf, void* ws) {
  uint8_t* w8 = (uint8_t*)ws;
  hs::SplitArgs sa;
  sa.A = A; sa.lda = lda; sa.B = B; sa.ldb = ldb;
  sa.m = (int32_t)p->m; sa.n = (int32_t)p->n; sa.k0 = (int32_t)k0; sa.w = (int32_t)(k1 - k0);
  const int64_t pad = p->fmt == 1 ? hs::kSplitChunk : 64;
  sa.Wp = (int32_t)(((k1 - k0) + pad - 1) / pad * pad);
  sa.fmt = p->fmt;
  sa.smax = p->opts.max_slices;
  sa.fixed_s = p->opts.slices; sa.smin = p->opts.min_slices; sa.tau_bits = p->opts.tau_bits;
  sa.log2k = (float)std::log2((double)std::max<int64_t>(1, p->k));
  sa.log2w = (float)std::log2((double)std::max<int64_t>(1, k1 - k0));
  sa.digA = w8 + (buf ? p->off_digA1 : p->off_digA); sa.planeA = (int64_t)p->m * sa.Wp;
  sa.digB = w8 + (buf ? p->off_digB1 : p->off_digB); sa.planeB = (int64_t)p->n * sa.Wp;
  sa.eA = (int32_t*)(w8 + (buf ? p->off_eA1 : p->off_eA));
  sa.fB = (int32_t*)(w8 + (buf ? p->off_fB1 : p->off_fB));
  sa.part = (double*)(w8 + (buf ? p->off_part1 : p->off_part));
  sa.nslab = (sa.Wp + 63) / 64;
  sa.stats = (uint32_t*)(w8 + p->off_stats) + hs::kStatWords * slot;
  sa.slices_out = (int32_t*)(w8 + p->off_slices) + slot;
  return sa;
}

// The panel pass of a precision form: clear the panel's statistics, then
// the statistics and digit kernels.
int launch_panel_split(const hs::SplitArgs& sa, hipStream_t stream) {
  hipError_t e = hs::launch_zero_u32(sa.stats, hs::kStatWords, stream);
  if (e != hipSuccess) {
    set_error(std::string("stats clear: ") + hipGetErrorString(e));
    return HSUMMA_ERR_DEVICE;
  }
  e = hs::launch_split(sa, stream);
  if (e != hipSuccess) {
    set_error(std::string("split launch: ") + hipGetErrorString(e));
    return HSUMMA_ERR_DEVICE;
  }
  return HSUMMA_OK;
}

// The product pass of a precision form over the panel split into `sa`: the
// slice products of every work item, then the FP64 route.
int launch_panel_products(hsumma_plan_t p, const hs::SplitArgs& sa, double* C, int64_t ldc,
                          int64_t k0, int64_t k1, int zero_init, void* ws, hipStream_t stream) {
  uint8_t* w8 = (uint8_t*)ws;
  int grid = 0;
  int rc = launch_grid(p, true, 1, &grid);
  if (rc) return rc;
  hs::SliceArgs la;
  la.digA = sa.digA; la.planeA = sa.planeA; la.rowsA = sa.m;
  la.digB = sa.digB; la.planeB = sa.planeB; la.rowsB = sa.n;
  {
    const int64_t esz = p->fmt == 0 ? 2 : 1;
    la.bytesA = (uint32_t)(p->opts.max_slices * sa.planeA * esz);
    la.bytesB = (uint32_t)(p->opts.max_slices * sa.planeB * esz);
  }
  la.eA = sa.eA; la.fB = sa.fB;
  la.slices = sa.slices_out;
  la.C = C; la.ldc = ldc;
  la.items = (const hs::WorkItem*)(w8 + p->off_items);
  la.nitems = (int32_t)p->items.size(); la.per_xcd = p->per_xcd;
  la.Wp = sa.Wp; la.nchunks = sa.Wp / hs::kSplitChunk;
  la.zero_init = zero_init; la.persistent = 1;
  la.dump = (double*)(w8 + p->off_dump);
  hipError_t e = hs::launch_slices(p->fmt, la, grid, stream);
  if (e != hipSuccess) {
    set_error(std::string("slice products launch: ") + hipGetErrorString(e));
    return HSUMMA_ERR_DEVICE;
  }
  // A panel the split cannot carry to FP64 accuracy (its modelled need is
  // beyond max_slices digits, or it holds a non-finite value) is computed by
  // the FP64 kernel instead, on the same items; the decision is on the device
  // (slice count 0), so both launches are always issued and exactly one of
  // them does work.
  return launch_fp64_range(p, hs::TileCfg{64, 128, 16}, sa.A, sa.lda, sa.B, sa.ldb, C, ldc, k0,
                           k1, zero_init, true, sa.slices_out, ws, stream);
}

// Launch the local update over k-range [k0, k1) (starting at an inner-step
// boundary) for every work item; the table must already be in `ws`.  `slot`
// indexes the per-panel statistics of the precision form.
int launch_range(hsumma_plan_t p, const double* A, int64_t lda, const double* B, int64_t ldb,
                 double* C, int64_t ldc, int64_t k0, int64_t k1, int zero_init, int64_t slot,
                 void* ws, hipStream_t stream, bool products_only = false) {
  if (p->items.empty()) return HSUMMA_OK;
  if (p->fmt < 0)
    return launch_fp64_range(p, p->cfg, A, lda, B, ldb, C, ldc, k0, k1, zero_init,
                             p->opts.persistent != 0, nullptr, ws, stream);
  // a look-ahead plan keeps outer panel g's planes in set g % 2 in every call
  const int buf = p->lookahead ? (int)(slot & 1) : 0;
  const hs::SplitArgs sa = split_args(p, A, lda, B, ldb, k0, k1, slot, buf, ws);
  if (!products_only) {
    int rc = launch_panel_split(sa, stream);
    if (rc) return rc;
  }
  return launch_panel_products(p, sa, C, ldc, k0, k1, zero_init, ws, stream);
}

// Whether a call overlaps the splits with the products: a look-ahead plan
// with more than one outer step; in the automatic mode (opts.lookahead = 2)
// only where one product launch has fewer work items than the device has
// CUs -- the split then runs on CUs the products leave idle, while where the
// persistent product launch holds every CU (its workgroups cannot share a
// CU with the split's) the overlap gained nothing and cost up to 1 %.
int lookahead_for_call(hsumma_plan_t p, bool* on) {
  *on = p->lookahead && p->outer_lo.size() > 2;
  if (!*on || p->opts.lookahead != 2) return HSUMMA_OK;
  int dev = 0, cus = 0;
  HS_CHECK_HIP(hipGetDevice(&dev));
  HS_CHECK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  *on = (int64_t)p->items.size() < (int64_t)cus;
  return HSUMMA_OK;
}

// The second stream and the events of a look-ahead plan, made on first use
// (the caller holds the plan's mutex); the plan then stays on that device.
int ensure_aux(hsumma_plan_t p) {
  int dev = 0;
  HS_CHECK_HIP(hipGetDevice(&dev));
  if (p->aux) {
    if (p->adevice != dev) return invalid("a plan with look-ahead is used on one device only");
    return HSUMMA_OK;
  }
  hipStream_t st = nullptr;
  HS_CHECK_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  for (int i = 0; i < 3; ++i) {
    const hipError_t e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
    if (e != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipEventDestroy(ev[j]);
      (void)hipStreamDestroy(st);
      set_error(std::string("look-ahead event: ") + hipGetErrorString(e));
      return HSUMMA_ERR_DEVICE;
    }
  }
  p->aux = st;
  p->ev_start = ev[0];
  p->ev_split = ev[1];
  p->ev_prod = ev[2];
  p->adevice = dev;
  return HSUMMA_OK;
}

// A named range per outer step (host side: it brackets the launches, which
// run asynchronously) for tools that trace roctx markers.
struct StepRange {
  explicit StepRange(int64_t g) {
    char name[48];
    std::snprintf(name, sizeof(name), "hsumma outer step %lld", (long long)g);
    roctxRangePushA(name);
  }
  ~StepRange() { roctxRangePop(); }
};

// The whole product of a split form with look-ahead (Sec. VI: the next
// step's panel work overlaps this step's update).  The split of panel g + 1
// runs on the plan's second stream, into the other digit-plane set, while
// the products of panel g run on the caller's stream.  Events order each
// split after the product pass that last read its set (panel g - 1) and
// each product pass after its split; every split is waited for by the
// caller's stream, so the call's work all ends there.  The kernels and
// their inputs are those of the plain sequence: the result is the same, bit
// for bit.
int run_lookahead(hsumma_plan_t p, const double* A, int64_t lda, const double* B, int64_t ldb,
                  double* C, int64_t ldc, void* ws, hipStream_t s) {
  int rc = prepare_items(p, ws, s);
  if (rc) return rc;
  const int64_t nouter = (int64_t)p->outer_lo.size() - 1;
  const int64_t* lo = p->outer_lo.data();
  HS_CHECK_HIP(hipEventRecord(p->ev_start, s));
  rc = launch_panel_split(split_args(p, A, lda, B, ldb, lo[0], lo[1], 0, 0, ws), s);
  if (rc) return rc;
  bool pending = false;   // a split on the second stream not yet waited for
  for (int64_t g = 0; g < nouter && !rc; ++g) {
    StepRange range(g);
    if (pending) {
      HS_CHECK_HIP(hipStreamWaitEvent(s, p->ev_split, 0));
      pending = false;
    }
    if (g + 1 < nouter) {
      HS_CHECK_HIP(hipStreamWaitEvent(p->aux, g == 0 ? p->ev_start : p->ev_prod, 0));
      rc = launch_panel_split(
          split_args(p, A, lda, B, ldb, lo[g + 1], lo[g + 2], g + 1, (int)((g + 1) & 1), ws),
          p->aux);
      HS_CHECK_HIP(hipEventRecord(p->ev_split, p->aux));
      pending = true;
      if (rc) break;
    }
    rc = launch_panel_products(p, split_args(p, A, lda, B, ldb, lo[g], lo[g + 1], g, (int)(g & 1), ws),
                               C, ldc, lo[g], lo[g + 1], g == 0 ? 1 : 0, ws, s);
    if (!rc) HS_CHECK_HIP(hipEventRecord(p->ev_prod, s));
  }
  // after an error too: nothing of this call stays on the second stream alone
  if (pending) HS_CHECK_HIP(hipStreamWaitEvent(s, p->ev_split, 0));
  return rc;
}

// The whole product: the work-item table, then every outer step in order
// (the first stores instead of accumulating).
int run_direct(hsumma_plan_t p, const double* A, int64_t lda, const double* B, int64_t ldb,
               double* C, int64_t ldc, void* ws, hipStream_t stream, bool lookahead) {
  if (lookahead) return run_lookahead(p, A, lda, B, ldb, C, ldc, ws, stream);
  int rc = prepare_items(p, ws, stream);
  if (rc) return rc;
  const int64_t nouter = (int64_t)p->outer_lo.size() - 1;
  for (int64_t g = 0; g < nouter; ++g) {
    StepRange range(g);
    rc = launch_range(p, A, lda, B, ldb, C, ldc, p->outer_lo[g], p->outer_lo[g + 1],
                      g == 0 ? 1 : 0, g, ws, stream);
    if (rc) return rc;
  }
  return HSUMMA_OK;
}

// run_direct for a caller's call: a look-ahead plan's second stream and
// events are shared by the plan's calls, so those calls are serialised.
int run_direct_call(hsumma_plan_t p, const double* A, int64_t lda, const double* B, int64_t ldb,
                    double* C, int64_t ldc, void* ws, hipStream_t s) {
  bool la = false;
  int rc = lookahead_for_call(p, &la);
  if (rc) return rc;
  if (!la) return run_direct(p, A, lda, B, ldb, C, ldc, ws, s, false);
  std::lock_guard<std::mutex> lk(p->mu);
  if ((rc = ensure_aux(p))) return rc;
  return run_direct(p, A, lda, B, ldb, C, ldc, ws, s, true);
}

// Whole product on an explicit workspace, direct or through the plan's graph.
int run_on(hsumma_plan_t p, const double* A, int64_t lda, const double* B, int64_t ldb,
           double* C, int64_t ldc, void* ws, hipStream_t s) {
  if (!p->opts.use_graph || s == nullptr) return run_direct_call(p, A, lda, B, ldb, C, ldc, ws, s);

  // Graph mode: capture the launch sequence (table generation included)
  // once per (pointers, stream, device) and replay it.  With look-ahead the
  // second stream joins the capture through the events and is joined back
  // before it ends.
  std::lock_guard<std::mutex> lk(p->mu);
  bool la = false;
  int rc0 = lookahead_for_call(p, &la);
  if (!rc0 && la) rc0 = ensure_aux(p);   // outside the capture
  if (rc0) return rc0;
  int dev = 0;
  HS_CHECK_HIP(hipGetDevice(&dev));
  GraphKey key{A, lda, B, ldb, C, ldc, ws, (void*)s};
  if (!(p->have_graph && p->gkey == key && p->gdevice == dev)) {
    if (p->gexec) {
      hipGraphExecDestroy(p->gexec);
      p->gexec = nullptr;
      p->have_graph = false;
    }
    HS_CHECK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc2 = run_direct(p, A, lda, B, ldb, C, ldc, ws, s, la);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (rc2) {
      if (graph) hipGraphDestroy(graph);
      return rc2;
    }
    if (e != hipSuccess) {
      set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      return HSUMMA_ERR_DEVICE;
    }
    e = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) {
      p->gexec = nullptr;
      set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
      return HSUMMA_ERR_DEVICE;
    }
    p->gkey = key;
    p->gdevice = dev;
    p->have_graph = true;
  }
  HS_CHECK_HIP(hipGraphLaunch(p->gexec, s));
  return HSUMMA_OK;
}

// ---- workspace for callers that cannot allocate ------------------------------
// A file-scope device array stands in for the caller's workspace in
// hsumma_run_noalloc.  Each device holds its own copy from the moment the
// library's code object is loaded on it until the process ends.  Host code
// must not use the array's name as an address: the device address is taken
// once per device with hipGetSymbolAddress (that device current) and used
// for every kernel argument.  Every call on one device shares the array, so
// such calls must not overlap on that device (they race); each call rewrites
// what it reads (work-item table, digit planes) and clears what must start
// at zero (the per-panel statistics, by kernel), so it does not depend on
// what an earlier call left there.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(4096) uint8_t scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // per device id; null until first use

int scratch_address(void** out) {
  int dev = 0;
  HS_CHECK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HS_CHECK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr || (((uintptr_t)ptr) & 255)) {
      set_error("scratch array: unexpected device address");
      return HSUMMA_ERR_DEVICE;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return HSUMMA_OK;
}

}  // namespace

extern "C" {

void hsumma_opts_default(hsumma_opts* o) {
  if (o) std::memset(o, 0, sizeof(*o));
}

const char* hsumma_last_error(void) { return hs::g_last_error.c_str(); }

const char* hsumma_version(void) { return "hsumma-gfx950 0.1"; }

int hsumma_plan(hsumma_plan_t* out, int64_t n, int32_t P, int32_t Q, int32_t G, int64_t b,
                int64_t M, const hsumma_opts* opts) {
  if (!out) return invalid("null output pointer");
  *out = nullptr;
  hsumma_opts o;
  hsumma_opts_default(&o);
  if (opts) o = *opts;
  const int64_t m = o.m ? o.m : n;
  const int64_t k = o.k ? o.k : n;
  if (n < 1 || m < 1 || k < 0 || o.m < 0 || o.k < 0) return invalid("matrix sizes must be positive");
  if (m >= (1LL << 31) || n >= (1LL << 31) || k >= (1LL << 31))
    return invalid("m, n and k must be below 2^31");
  if (P < 1 || Q < 1) return invalid("P and Q must be >= 1");
  if (P > m || Q > n) return invalid("grid larger than the matrix (need P <= m, Q <= n)");
  if (G < 1) return invalid("G must be >= 1");
  if (b < 1) return invalid("b must be >= 1");
  if (M < b) return invalid("outer block M must be >= inner block b");
  if (M % b) return invalid("outer block M must be a multiple of b");
  if (o.dist != HSUMMA_DIST_BLOCK && o.dist != HSUMMA_DIST_BLOCK_CYCLIC)
    return invalid("unknown distribution");
  if (o.prec != HSUMMA_FP64 && o.prec != HSUMMA_SPLIT_BF16 && o.prec != HSUMMA_SPLIT_FP8 &&
      o.prec != HSUMMA_SPLIT_INT8)
    return invalid("unknown precision");
  if (o.nb < 0) return invalid("nb must be >= 0");
  if (o.wgs_per_cu < 0) return invalid("wgs_per_cu must be >= 0");
  if (o.lookahead < 0 || o.lookahead > 2) return invalid("lookahead must be 0, 1 or 2");
  int I = 0, J = 0;
  if (!hs::factor_groups(P, Q, G, &I, &J))
    return invalid("G cannot be arranged as I x J groups with I | P and J | Q");

  hsumma_plan_s* p = new (std::nothrow) hsumma_plan_s();
  if (!p) return invalid("out of host memory");
  p->m = m; p->n = n; p->k = k; p->b = b; p->M = M;
  p->nb = o.nb ? o.nb : b;
  p->P = P; p->Q = Q; p->G = G; p->I = I; p->J = J;
  p->opts = o;
  p->opts.m = m; p->opts.k = k; p->opts.nb = p->nb;
  p->rlo = block_bounds(m, P);
  p->clo = block_bounds(n, Q);

  // Tile configuration.
  if (o.prec == HSUMMA_FP64) {
    hs::TileCfg cfg{o.tile_m ? o.tile_m : 128, o.tile_n ? o.tile_n : 128, o.kc ? o.kc : 16,
                    o.waves};
    if (!o.tile_m && !o.tile_n && !o.kc) {
      const hs::TileCfg d = default_tile(*p);
      cfg = {d.tm, d.tn, d.kc, o.waves};
    } else if (!o.tile_m && !o.tile_n && (m < 512 || n < 512)) {
      cfg = {64, 64, o.kc, o.waves};
    }
    bool ok = false;
    for (auto& c : hs::fp64_configs())
      if (hs::same_tile(cfg, c)) {
        ok = true;
        cfg.waves = c.waves;           // the first compiled configuration of the tile
        break;
      }
    if (!ok) {
      delete p;
      return invalid("tile configuration (tile_m, tile_n, kc, waves) not compiled into the library");
    }
    p->cfg = cfg;
  } else {
    p->fmt = o.prec == HSUMMA_SPLIT_BF16 ? 0 : o.prec == HSUMMA_SPLIT_FP8 ? 1 : 2;
    // every form: 64 x 128 macro-tiles streamed in 16-k steps (32-k for INT8)
    const hs::TileCfg scfg{64, 128, p->fmt == 2 ? 32 : 16};
    if ((o.tile_m && o.tile_m != scfg.tm) || (o.tile_n && o.tile_n != scfg.tn) ||
        (o.kc && o.kc != scfg.kc) || (o.waves && o.waves != 4)) {
      delete p;
      return invalid("split forms use fixed 64 x 128 macro-tiles and 16-k steps (32-k for INT8)");
    }
    p->cfg = scfg;
    const int slim = hs::split_max_slices(p->fmt);
    if (!p->opts.min_slices) p->opts.min_slices = 3;
    if (!p->opts.max_slices) p->opts.max_slices = slim;
    // INT8 digits drop more of the product at a given bit count than BF16
    // ones (more, larger digit pairs beyond the kept levels): two more bits
    if (!p->opts.tau_bits) p->opts.tau_bits = p->fmt == 2 ? 50 : 48;
    const int smin = p->opts.min_slices, smax = p->opts.max_slices, sf = p->opts.slices;
    if (smin < 1 || smax > slim || smin > smax || sf < 0 || sf > slim) {
      delete p;
      return invalid(slim == 8 ? "slice counts must satisfy 1 <= min_slices <= max_slices <= 8, slices <= 8"
                               : "slice counts must satisfy 1 <= min_slices <= max_slices <= 7, slices <= 7");
    }
    if (sf > smax) p->opts.max_slices = sf;
    if (p->fmt == 1 && M > 8192) {
      delete p;
      return invalid("FP8 split form needs M <= 8192 (exact FP32 accumulation over a panel)");
    }
    if (p->fmt == 2 && M > 8192) {
      delete p;
      return invalid("INT8 split form needs M <= 8192 (exact INT32 accumulation over a panel)");
    }
    // BF16 steps in groups of 64 k, INT8 in pairs of 32-k steps
    const int64_t pad = p->fmt == 1 ? hs::kSplitChunk : 64;
    const int64_t Wp = (M + pad - 1) / pad * pad;
    if ((Wp + 63) / 64 > 65535) {
      delete p;
      return invalid("split forms need an outer block M of at most 4194240 (the split kernels "
                     "take one grid row per 64 columns of the panel, at most 65535)");
    }
    p->Wp = (int32_t)Wp;
    const int64_t esz = p->fmt == 0 ? 2 : 1;
    // the slice kernels address each operand's digit planes through a buffer
    // descriptor with 32-bit offsets
    if (p->opts.max_slices * std::max(m, n) * Wp * esz > (int64_t)0xFFFFFFFF) {
      delete p;
      return invalid("split form: the digit planes of one operand panel exceed 4 GiB "
                     "(max_slices x rows x padded M x digit bytes); use a smaller outer block M");
    }
  }

  p->kqlo = block_bounds(k, Q);
  p->kplo = block_bounds(k, P);
  for (int64_t g0 = 0; g0 < k; g0 += M) {
    const int64_t g1 = std::min(g0 + M, k);
    p->outer_lo.push_back(g0);
    for (int64_t s0 = g0; s0 < g1; s0 += b)
      p->steps.push_back({s0, std::min(s0 + b, g1), (int64_t)p->outer_lo.size() - 1});
  }
  p->outer_lo.push_back(k);
  if (k == 0) p->outer_lo.assign(1, 0);
  if ((int64_t)P * Q > hs::kGenMaxProcs) {
    delete p;
    return invalid("grid of more than " + std::to_string(hs::kGenMaxProcs) +
                   " virtual processors (the work-item generator keeps one count per "
                   "processor on chip)");
  }
  int64_t max_row_block = 0;
  build_items(*p, &max_row_block);
  if (p->items.size() > (size_t)0x7FFFF000 || max_row_block >= (int64_t(1) << 31)) {
    delete p;
    return invalid("more than 2^31 work items (use larger macro-tiles or a smaller problem)");
  }
  // Workspace layout: the work-item table (and, for the longest-first order,
  // its unordered copy), then the precision form's digit planes, exponents,
  // per-slab partial statistics, per-panel statistics and slice counts, and
  // the INT8 kernel's dump area (with look-ahead, a second set of planes,
  // exponents and partial statistics after it).
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  // the digit planes and partial statistics start on 4 KiB boundaries of the
  // workspace: with a 4 KiB-aligned workspace the product kernels' 1 KB DMA
  // runs then stay inside aligned 4 KiB units (measured: a workspace 256 or
  // 1536 bytes off a 4 KiB boundary made the INT8 product kernel 1.7 %
  // slower)
  auto al4k = [](size_t x) { return (x + 4095) & ~(size_t)4095; };
  size_t off = 0;
  const size_t nit = p->items.size();
  p->off_items = off; off = al(off + nit * sizeof(hs::WorkItem));
  p->off_items_tmp = off; if (p->lpt) off = al(off + nit * sizeof(hs::WorkItem));
  if (p->fmt >= 0) {
    const size_t esz = p->fmt == 0 ? 2 : 1;
    const size_t Wp = (size_t)p->Wp, sl = (size_t)p->opts.max_slices;
    const size_t nout = (size_t)std::max<int64_t>(1, (k + M - 1) / M);
    p->off_digA = off = al4k(off); off = al(off + sl * (size_t)m * Wp * esz);
    p->off_digB = off = al4k(off); off = al(off + sl * (size_t)n * Wp * esz);
    p->off_eA = off; off = al(off + (size_t)m * 4);
    p->off_fB = off; off = al(off + (size_t)n * 4);
    p->off_part = off = al4k(off); off = al(off + (size_t)hs::split_part_doubles(m, n, p->Wp) * 8);
    p->off_stats = off; off = al(off + nout * hs::kStatWords * 4);
    p->off_slices = off; off = al(off + nout * 4);
    p->off_dump = off; off = al(off + 64 * sizeof(double));
    if (o.lookahead) {
      p->lookahead = true;
      p->off_digA1 = off = al4k(off); off = al(off + sl * (size_t)m * Wp * esz);
      p->off_digB1 = off = al4k(off); off = al(off + sl * (size_t)n * Wp * esz);
      p->off_eA1 = off; off = al(off + (size_t)m * 4);
      p->off_fB1 = off; off = al(off + (size_t)n * 4);
      p->off_part1 = off = al4k(off); off = al(off + (size_t)hs::split_part_doubles(m, n, p->Wp) * 8);
    }
  }
  p->ws_bytes = std::max<size_t>(off, 256);
  *out = p;
  return HSUMMA_OK;
}

void hsumma_plan_destroy(hsumma_plan_t p) {
  if (!p) return;
  if (p->gexec) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) cur = -1;
    if (p->gdevice >= 0 && p->gdevice != cur) hipSetDevice(p->gdevice);
    hipGraphExecDestroy(p->gexec);
    if (cur >= 0 && p->gdevice != cur) hipSetDevice(cur);
  }
  if (p->aux) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) cur = -1;
    if (p->adevice >= 0 && p->adevice != cur) hipSetDevice(p->adevice);
    // the calls that used the second stream joined it into their own
    // stream; its last work must still end before the stream goes
    (void)hipStreamSynchronize(p->aux);
    (void)hipEventDestroy(p->ev_start);
    (void)hipEventDestroy(p->ev_split);
    (void)hipEventDestroy(p->ev_prod);
    (void)hipStreamDestroy(p->aux);
    if (cur >= 0 && p->adevice != cur) hipSetDevice(cur);
  }
  delete p;
}

int hsumma_workspace_size(hsumma_plan_t p, size_t* bytes) {
  if (!p || !bytes) return invalid("null argument");
  *bytes = p->ws_bytes;
  return HSUMMA_OK;
}

int hsumma_num_steps(hsumma_plan_t p, int64_t* steps) {
  if (!p || !steps) return invalid("null argument");
  *steps = (int64_t)p->steps.size();
  return HSUMMA_OK;
}

int hsumma_num_outer_steps(hsumma_plan_t p, int64_t* steps) {
  if (!p || !steps) return invalid("null argument");
  *steps = (int64_t)p->outer_lo.size() - 1;
  return HSUMMA_OK;
}

int hsumma_groups(hsumma_plan_t p, int32_t* I, int32_t* J) {
  if (!p || !I || !J) return invalid("null argument");
  *I = p->I;
  *J = p->J;
  return HSUMMA_OK;
}

int hsumma_tile_config(hsumma_plan_t p, int32_t* tile_m, int32_t* tile_n, int32_t* kc,
                       int32_t* waves) {
  if (!p || !tile_m || !tile_n || !kc || !waves) return invalid("null argument");
  *tile_m = p->cfg.tm;
  *tile_n = p->cfg.tn;
  *kc = p->cfg.kc;
  *waves = p->fmt < 0 ? p->cfg.waves : 4;
  return HSUMMA_OK;
}

int hsumma_num_items(hsumma_plan_t p, int64_t* items) {
  if (!p || !items) return invalid("null argument");
  *items = (int64_t)p->items.size();
  return HSUMMA_OK;
}

int hsumma_tile_shape(hsumma_plan_t p, int32_t pr, int32_t pc, int64_t* m_loc, int64_t* n_loc) {
  if (!p || !m_loc || !n_loc) return invalid("null argument");
  if (pr < 0 || pr >= p->P || pc < 0 || pc >= p->Q) return invalid("processor index out of range");
  *m_loc = local_count(*p, true, pr);
  *n_loc = local_count(*p, false, pc);
  return HSUMMA_OK;
}

int hsumma_step_info(hsumma_plan_t p, int64_t s, int64_t* k0, int64_t* k1, int64_t* outer,
                     int32_t* owner_col, int32_t* owner_row, int32_t* group_col,
                     int32_t* group_row, int32_t* in_group_col, int32_t* in_group_row) {
  if (!p) return invalid("null plan");
  if (s < 0 || s >= (int64_t)p->steps.size()) return invalid("step out of range");
  const StepRec& st = p->steps[s];
  int q, r;
  if (p->opts.dist == HSUMMA_DIST_BLOCK) {
    q = owner_block(p->kqlo, st.k0);
    r = owner_block(p->kplo, st.k0);
  } else {
    q = (int)((st.k0 / p->nb) % p->Q);
    r = (int)((st.k0 / p->nb) % p->P);
  }
  const int gq = p->Q / p->J, gp = p->P / p->I;
  if (k0) *k0 = st.k0;
  if (k1) *k1 = st.k1;
  if (outer) *outer = st.outer;
  if (owner_col) *owner_col = q;
  if (owner_row) *owner_row = r;
  if (group_col) *group_col = q / gq;
  if (group_row) *group_row = r / gp;
  if (in_group_col) *in_group_col = q % gq;
  if (in_group_row) *in_group_row = r % gp;
  return HSUMMA_OK;
}

int hsumma_local_update(hsumma_plan_t p, int64_t step, const double* A, int64_t lda,
                        const double* B, int64_t ldb, double* C, int64_t ldc, void* ws,
                        size_t ws_bytes, void* stream) {
  int rc = check_operands(p, A, lda, B, ldb, C, ldc);
  if (rc) return rc;
  if (step < 0 || step >= (int64_t)p->steps.size()) return invalid("step out of range");
  if ((rc = check_ws(p, ws, ws_bytes))) return rc;
  if ((rc = prepare_items(p, ws, (hipStream_t)stream))) return rc;
  const StepRec& st = p->steps[step];
  return launch_range(p, A, lda, B, ldb, C, ldc, st.k0, st.k1, 0, st.outer, ws,
                      (hipStream_t)stream);
}

int hsumma_outer_update(hsumma_plan_t p, int64_t outer, const double* A, int64_t lda,
                        const double* B, int64_t ldb, double* C, int64_t ldc, void* ws,
                        size_t ws_bytes, void* stream) {
  int rc = check_operands(p, A, lda, B, ldb, C, ldc);
  if (rc) return rc;
  if (outer < 0 || outer >= (int64_t)p->outer_lo.size() - 1) return invalid("outer step out of range");
  if ((rc = check_ws(p, ws, ws_bytes))) return rc;
  StepRange range(outer);
  if ((rc = prepare_items(p, ws, (hipStream_t)stream))) return rc;
  return launch_range(p, A, lda, B, ldb, C, ldc, p->outer_lo[outer], p->outer_lo[outer + 1], 0,
                      outer, ws, (hipStream_t)stream);
}

int hsumma_outer_products(hsumma_plan_t p, int64_t outer, const double* A, int64_t lda,
                          const double* B, int64_t ldb, double* C, int64_t ldc, void* ws,
                          size_t ws_bytes, void* stream) {
  if (!p) return invalid("null plan");
  if (p->fmt < 0) {
    set_error("hsumma_outer_products is for the split forms");
    return HSUMMA_ERR_UNSUPPORTED;
  }
  int rc = check_operands(p, A, lda, B, ldb, C, ldc);
  if (rc) return rc;
  if (outer < 0 || outer >= (int64_t)p->outer_lo.size() - 1) return invalid("outer step out of range");
  if ((rc = check_ws(p, ws, ws_bytes))) return rc;
  if ((rc = prepare_items(p, ws, (hipStream_t)stream))) return rc;
  return launch_range(p, A, lda, B, ldb, C, ldc, p->outer_lo[outer], p->outer_lo[outer + 1], 0,
                      outer, ws, (hipStream_t)stream, true);
}

int hsumma_run(hsumma_plan_t p, const double* A, int64_t lda, const double* B, int64_t ldb,
               double* C, int64_t ldc, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_operands(p, A, lda, B, ldb, C, ldc);
  if (rc) return rc;
  if ((rc = check_ws(p, ws, ws_bytes))) return rc;
  return run_on(p, A, lda, B, ldb, C, ldc, ws, (hipStream_t)stream);
}

int hsumma_run_noalloc(hsumma_plan_t p, const double* A, int64_t lda, const double* B,
                       int64_t ldb, double* C, int64_t ldc, void* stream) {
  int rc = check_operands(p, A, lda, B, ldb, C, ldc);
  if (rc) return rc;
  if (p->ws_bytes > kScratchBytes) {
    set_error("hsumma_run_noalloc: the plan needs " + std::to_string(p->ws_bytes) +
              " bytes of workspace, more than the library's " +
              std::to_string(kScratchBytes) + "-byte scratch array; use hsumma_run");
    return HSUMMA_ERR_WORKSPACE;
  }
  void* ws = nullptr;
  if ((rc = scratch_address(&ws))) return rc;
  return run_direct_call(p, A, lda, B, ldb, C, ldc, ws, (hipStream_t)stream);
}

size_t hsumma_noalloc_max_workspace(void) { return kScratchBytes; }

int hsumma_prepare_workspace(hsumma_plan_t p, void* ws, size_t ws_bytes, void* stream) {
  if (!p) return invalid("null plan");
  int rc = check_ws(p, ws, ws_bytes);
  if (rc) return rc;
  return prepare_items(p, ws, (hipStream_t)stream);
}

int hsumma_work_items(hsumma_plan_t p, int32_t* out, int64_t capacity) {
  if (!p || !out) return invalid("null argument");
  if (capacity < (int64_t)p->items.size()) return invalid("output smaller than hsumma_num_items()");
  for (size_t i = 0; i < p->items.size(); ++i) {
    out[4 * i + 0] = p->items[i].r0;
    out[4 * i + 1] = p->items[i].c0;
    out[4 * i + 2] = p->items[i].h;
    out[4 * i + 3] = p->items[i].w;
  }
  return HSUMMA_OK;
}

int hsumma_panel_slices(hsumma_plan_t p, const void* ws, int32_t* counts, void* stream) {
  if (!p || !counts) return invalid("null argument");
  if (p->fmt < 0) {
    set_error("the FP64 path has no slices");
    return HSUMMA_ERR_UNSUPPORTED;
  }
  if (!ws) return invalid("null workspace");
  const int64_t nout = (int64_t)p->outer_lo.size() - 1;
  hipStream_t s = (hipStream_t)stream;
  HS_CHECK_HIP(hipMemcpyAsync(counts, (const uint8_t*)ws + p->off_slices, (size_t)nout * 4,
                              hipMemcpyDeviceToHost, s));
  HS_CHECK_HIP(hipStreamSynchronize(s));
  return HSUMMA_OK;
}

int hsumma_split_layout(hsumma_plan_t p, size_t* off_digA, size_t* off_digB, size_t* off_eA,
                        size_t* off_fB, int32_t* Wp, int32_t* planes) {
  if (!p) return invalid("null plan");
  if (p->fmt < 0) {
    set_error("the FP64 path has no split workspace");
    return HSUMMA_ERR_UNSUPPORTED;
  }
  if (off_digA) *off_digA = p->off_digA;
  if (off_digB) *off_digB = p->off_digB;
  if (off_eA) *off_eA = p->off_eA;
  if (off_fB) *off_fB = p->off_fB;
  if (Wp) *Wp = p->Wp;
  if (planes) *planes = p->opts.max_slices;
  return HSUMMA_OK;
}

int hsumma_mfma_exact_probe(int32_t fmt, const void* a, const void* b, int32_t k, float* d,
                            void* stream) {
  if (fmt != 0 && fmt != 1 && fmt != 2) return invalid("fmt must be 0 (BF16), 1 (FP8-e4m3) or 2 (INT8)");
  if (!a || !b || !d) return invalid("null pointer");
  if (fmt == 2 ? (k < 32 || k % 32) : (k < 16 || k % 16))
    return invalid("k must be a positive multiple of 16 (32 for INT8)");
  hipError_t e = hs::launch_mfma_probe(fmt, a, b, k, d, (hipStream_t)stream);
  if (e != hipSuccess) {
    set_error(std::string("probe launch: ") + hipGetErrorString(e));
    return HSUMMA_ERR_DEVICE;
  }
  return HSUMMA_OK;
}

}  // extern "C"
