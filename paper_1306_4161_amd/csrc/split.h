// Internal interface of the precision-form kernels (digit split + slice products).
#pragma once

#include "internal.h"

namespace hs {

constexpr int kSplitMaxSlices = 8;   // digit planes written per operand (any format)
// largest slice count of a format: 7 BF16 / FP8 digits, 8 INT8 digits
constexpr int split_max_slices(int fmt) { return fmt == 2 ? 8 : 7; }
constexpr int kSplitChunk = 32;      // panel width is padded to a multiple of this

// Per-panel statistics (uint32 words): the non-finite flag written by the
// statistics kernel, the maxima by the combine kernel:
constexpr int kStatKappaA = 0;       // max over A rows of log2 kappa (float bits)
constexpr int kStatKappaB = 1;       // max over B columns of log2 kappa (float bits)
constexpr int kStatCohA = 2;         // max over A rows of the residual coherence (float bits)
constexpr int kStatCohB = 3;         // max over B columns of the same
constexpr int kStatNonFinite = 4;    // nonzero if the panel holds an Inf or a NaN
constexpr int kStatLamA = 5;         // max over A rows of log2 max|x| - mean log2|x| (float bits)
constexpr int kStatLamB = 6;         // max over B columns of the same
constexpr int kStatWords = 8;        // words per panel (padded)

struct SplitArgs {
  const double* A; int64_t lda;      // panel = A(:, k0:k0+w)
  const double* B; int64_t ldb;      // panel = B(k0:k0+w, :)
  int32_t m, n, k0, w, Wp;           // Wp: padded panel width (multiple of kSplitChunk)
  int32_t fmt;                       // 0: BF16 digits, 1: FP8-e4m3 digits, 2: INT8 digits
  int32_t smax;                      // planes to write
  void* digA; int64_t planeA;        // planes of m x Wp digits (elements per plane)
  void* digB; int64_t planeB;        // planes of n x Wp digits (B transposed)
  int32_t* eA; int32_t* fB;          // per-row / per-column exponents
  uint32_t* stats;                   // kStatWords words, cleared before the statistics kernel
  double* part;                      // per-slab partial sums of every line (split_part_doubles)
  int32_t nslab;                     // 64-k slabs of the padded panel: ceil(Wp / 64)
  int32_t* slices_out;               // the panel's slice count (0: the FP64 kernel computes it)
  int32_t fixed_s, smin, tau_bits;   // slice-count choice: fixed count, bounds, target bits
  float log2k;                       // log2 of the product's inner dimension k
  float log2w;                       // log2 of the panel width
};

struct SliceArgs {
  const void* digA; int64_t planeA; int32_t rowsA;   // rowsA = m
  const void* digB; int64_t planeB; int32_t rowsB;   // rowsB = n
  uint32_t bytesA, bytesB;           // byte sizes of the two digit regions (< 4 GiB)
  const int32_t* eA; const int32_t* fB;
  const int32_t* slices;             // the panel's slice count, written by the digit kernel
                                     // (0: the launch does nothing)
  double* C; int64_t ldc;
  const WorkItem* items; int32_t nitems; int32_t per_xcd;
  int32_t Wp, nchunks;
  int32_t zero_init, persistent;
  double* dump;                      // 64 doubles of workspace: INT8 stores of lanes outside an item
};

// Doubles of the per-slab partial statistics of a panel of padded width Wp
// over m + n lines.
constexpr int64_t split_part_doubles(int64_t m, int64_t n, int64_t Wp) {
  return 6 * ((Wp + 63) / 64) * (m + n);
}

// Statistics pass (per-slab partial sums), their combination (exponents,
// kappa and the other panel statistics), then the digit pass, which writes
// only the panel's chosen number of planes.
hipError_t launch_split(const SplitArgs& a, hipStream_t s);
hipError_t launch_slices(int fmt, const SliceArgs& a, int grid, hipStream_t s);
hipError_t launch_zero_u32(uint32_t* p, int n, hipStream_t s);
hipError_t launch_mfma_probe(int fmt, const void* a, const void* b, int k, float* out,
                             hipStream_t s);

}  // namespace hs
