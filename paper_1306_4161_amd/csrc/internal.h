// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/hsumma.h"

namespace hs {

// One rectangle of C that one workgroup updates: rows [r0, r0+h) and
// columns [c0, c0+w) of the global row-major matrix.  It lies inside one
// virtual processor's tile (and, for the block-cyclic distribution, inside
// one distribution block), so it is a macro-tile of that processor's local
// update.
struct WorkItem {
  int32_t r0, c0, h, w;
};

// Arguments common to the update kernels of one launch.
struct UpdateArgs {
  const double* A; int64_t lda;
  const double* B; int64_t ldb;
  double* C; int64_t ldc;
  const WorkItem* items; int32_t nitems; int32_t per_xcd;
  int64_t k0, k1;      // k-range of this launch (starts at a step boundary)
  int64_t bstep;       // inner block b: quads restart at every step start
  int32_t zero_init;   // 1: start from C = 0 instead of loading C
  int32_t persistent;  // 1: grid-stride over the items (grouped persistent mode)
  const int32_t* gate; // non-null: the launch does nothing unless *gate == 0 (the
                       // split forms' FP64 route for a panel they cannot split)
  // items == nullptr: the items are the macro-tiles of one dense
  // dense_m x dense_n block of C, row-major over dense_nc tile columns
  // (dense_items1 of them), then those of a second block of dense_m2 x
  // dense_n2 right of it (columns dense_n .. dense_n + dense_n2, the same
  // rows of A from row 0), row-major over dense_nc2 tile columns
  int32_t dense_m, dense_n, dense_nc, dense_items1;
  int32_t dense_m2, dense_n2, dense_nc2;
};

// Parameters of the device-side work-item generator (k_items.hip), which
// keeps one prefix sum per virtual processor in LDS.
constexpr int kGenMaxProcs = 16384;
struct ItemGenArgs {
  int64_t m, n;            // rows and columns of C
  int32_t P, Q, I, J;      // grid and group arrangement
  int32_t tm, tn;          // macro-tile
  int32_t br, bc;          // macro-tiles per block inside a processor's tile
  int32_t dist;            // hsumma_dist
  int64_t nb;              // block-cyclic block
  int32_t nitems, per_xcd;
  int32_t lpt;             // 1: each XCD list in longest-first order
  WorkItem* items;         // the table (nitems)
  WorkItem* tmp;           // unordered items (nitems; used when lpt)
};
hipError_t launch_gen_items(const ItemGenArgs& g, hipStream_t s);

// Workgroup barrier of an LDS ring filled by direct-to-LDS loads.  Each wave
// first waits (s_waitcnt vmcnt) for its own loads of the stage it is about to
// read; __syncthreads() would add a release fence, i.e. a wait for every
// outstanding load, including those of later stages that are meant to stay in
// flight across the barrier.  lgkmcnt(0) retires this wave's LDS reads of the
// stage that is refilled next; the "memory" clobber keeps the compiler from
// moving LDS accesses across the barrier.
__device__ __forceinline__ void ring_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Buffer descriptor word 3 for raw (untyped) buffer loads on CDNA: data
// format 32 bits, no swizzle, no index stride.
constexpr int kBufferWord3 = 0x00020000;

// Kernel configurations (macro-tile, k-chunk, waves per workgroup) compiled
// into the library; waves = 0 selects the first configuration of that tile.
struct TileCfg {
  int tm, tn, kc;
  int waves = 0;
};
inline bool same_tile(const TileCfg& want, const TileCfg& have) {
  return want.tm == have.tm && want.tn == have.tn && want.kc == have.kc &&
         (want.waves == 0 || want.waves == have.waves);
}
const std::vector<TileCfg>& fp64_configs();
// dma: use the direct-to-LDS kernel of this configuration if there is one
// (the caller guarantees 16-byte granularity of every k-range and column run)
hipError_t launch_fp64(const TileCfg& cfg, const UpdateArgs& a, int grid, hipStream_t s,
                       bool dma);
bool fp64_has_dma(const TileCfg& cfg);
// C (m x n, ldc) += A (m x k) B (k x n) by the FP64 update kernel over the
// macro-tiles of C in row-major order (no work-item table): for updates of
// one dense block, e.g. inside an LU panel.  With m2, n2 > 0 the same launch
// also updates the block of rows [0, m2) and columns [n, n + n2) (B and C
// then have n + n2 columns): the L-shaped update of an LU panel step.
hipError_t launch_fp64_dense(const double* A, int64_t lda, const double* B, int64_t ldb,
                             double* C, int64_t ldc, int64_t m, int64_t n, int64_t k,
                             hipStream_t s, int64_t m2 = 0, int64_t n2 = 0);
int fp64_occupancy(const TileCfg& cfg);  // workgroups per CU the config is built for

// Split (precision) path.
struct SplitArgs;
struct SliceArgs;

void set_error(const std::string& msg);
// Most square I x J = G with I | P and J | Q (ties to the smaller I).
bool factor_groups(int P, int Q, int G, int* I, int* J);

}  // namespace hs
