// FP64 MFMA local update (the DGemm of Alg. 1) for gfx950.
//
// One workgroup owns one macro-tile of C (a WorkItem): it loads the C
// macro-tile into v_mfma_f64_16x16x4_f64 accumulators once, streams the
// launch's k-range through LDS in KC-deep chunks (double buffered, one
// barrier per chunk), and stores C once.  The k-range of a launch is one
// inner step (hsumma_local_update) or all inner steps of an outer step
// (hsumma_outer_update / hsumma_run); the 4-deep MFMA k-groups restart at
// every inner-step boundary, so both give bitwise identical results.
//
// MFMA operand layout (16x16x4, FP64, wave64), measured on gfx950:
//   A fragment: lane l holds A[l % 16][l / 16]  (16 x 4 block)
//   B fragment: lane l holds B[l / 16][l % 16]  (4 x 16 block)
//   D:          lane l, item v holds D[4 * v + l / 16][l % 16]
//
// LDS layouts (doubles):
//   As[row][k] with row stride KC + 1: the 16 rows x 4 k of an A fragment
//      fall on distinct banks.
//   Bs[k][col] with row stride TN + 16: the 4 k-rows of a B fragment are
//      half a bank-cycle apart.
//
// Global loads: every thread reads the same (row, k) pattern of each chunk
// from uniform per-chunk base addresses.  Full chunks of full macro-tiles
// take an unpredicated path; ragged edges (tile boundaries, the ragged last
// inner step) a predicated one that zero-fills.
#include <type_traits>

#include "internal.h"

namespace hs {

typedef double d4 __attribute__((ext_vector_type(4)));

template <int TM, int TN, int KC, int WM, int WN>
struct Fp64Tile {
  static constexpr int NT = WM * WN * 64;          // threads
  static constexpr int WTM = TM / WM;              // wave tile rows
  static constexpr int WTN = TN / WN;              // wave tile cols
  static constexpr int FM = WTM / 16;              // MFMA blocks per wave (rows)
  static constexpr int FN = WTN / 16;              // MFMA blocks per wave (cols)
  static constexpr int ASTR = KC + 1;              // As row stride
  static constexpr int BSTR = TN + 16;             // Bs row stride
  static constexpr int AS = TM * ASTR;             // doubles per A buffer
  static constexpr int BS = KC * BSTR;             // doubles per B buffer
  static constexpr int ALD = TM * KC / NT;         // A loads per thread per chunk
  static constexpr int BLD = TN * KC / NT;         // B loads per thread per chunk
  static constexpr int AROWS = NT / KC;            // A rows covered per load round
  static constexpr int BROWS = NT / TN;            // B k-rows covered per load round
  static_assert(TM % (WM * 16) == 0 && TN % (WN * 16) == 0, "wave tiling");
  static_assert((TM * KC) % NT == 0 && (TN * KC) % NT == 0, "load tiling");
  static_assert(NT % KC == 0 && NT % TN == 0, "load mapping");
  static_assert(KC % 4 == 0, "chunk is whole MFMA k-groups");
};

// Work item idx: from the table, or the idx-th macro-tile (row-major) of
// the dense block(s) when there is no table.
template <int TM, int TN>
__device__ __forceinline__ WorkItem fetch_item(const UpdateArgs& p, int idx) {
  if (p.items) return p.items[idx];
  if (idx < p.dense_items1) {
    const int tr = idx / p.dense_nc, tc = idx - tr * p.dense_nc;
    return WorkItem{tr * TM, tc * TN, min(TM, p.dense_m - tr * TM), min(TN, p.dense_n - tc * TN)};
  }
  idx -= p.dense_items1;
  const int tr = idx / p.dense_nc2, tc = idx - tr * p.dense_nc2;
  return WorkItem{tr * TM, p.dense_n + tc * TN, min(TM, p.dense_m2 - tr * TM),
                  min(TN, p.dense_n2 - tc * TN)};
}

template <int TM, int TN, int KC, int WM, int WN, int OCC>
__global__ __launch_bounds__(WM * WN * 64, OCC)
void fp64_update_kernel(UpdateArgs p) {
  using T = Fp64Tile<TM, TN, KC, WM, WN>;
  __shared__ double smem[2 * (T::AS + T::BS)];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int l16 = lane & 15, lq = lane >> 4;
  // this thread's load coordinates inside a chunk
  const int a_row = tid / KC, a_kk = tid % KC;
  const int b_kk = tid / TN, b_col = tid % TN;

  const int k0 = (int)p.k0, k1 = (int)p.k1, bstep = (int)p.bstep;
  if (p.gate && *p.gate != 0) return;

  const int bid = blockIdx.x;
  const int xcd = bid & 7;
  const int slot0 = bid >> 3;
  const int slots = p.persistent ? (gridDim.x + 7 - xcd) >> 3 : 1;

  for (int slot = slot0;; slot += slots) {
    if (!p.persistent && slot != slot0) break;
    if (slot >= p.per_xcd) break;
    const int idx = xcd * p.per_xcd + slot;
    if (idx >= p.nitems) break;
    const WorkItem it = fetch_item<TM, TN>(p, idx);
    const bool full_tile = (it.h == TM) && (it.w == TN);
    const double* __restrict__ Ab = p.A + (int64_t)it.r0 * p.lda;
    const double* __restrict__ Bb = p.B + it.c0;
    double* __restrict__ Cb = p.C + (int64_t)it.r0 * p.ldc + it.c0;

    d4 acc[T::FM][T::FN];
    // ---- load C (or start from zero) --------------------------------------
#pragma unroll
    for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < T::FN; ++fn)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[fm][fn][v] = 0.0;
    if (!p.zero_init) {
#pragma unroll
      for (int fm = 0; fm < T::FM; ++fm) {
#pragma unroll
        for (int fn = 0; fn < T::FN; ++fn) {
          const int col = wn * T::WTN + fn * 16 + l16;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = wm * T::WTM + fm * 16 + 4 * v + lq;
            if (full_tile || (row < it.h && col < it.w))
              acc[fm][fn][v] = Cb[(int64_t)row * p.ldc + col];
          }
        }
      }
    }

    double ra[T::ALD], rb[T::BLD];
    auto load_chunk = [&](int c0, int clen) {
      const double* Ac = Ab + c0;
      const double* Bc = Bb + (int64_t)c0 * p.ldb;
      if (full_tile && clen == KC) {
#pragma unroll
        for (int i = 0; i < T::ALD; ++i)
          ra[i] = Ac[(int64_t)(a_row + i * T::AROWS) * p.lda + a_kk];
#pragma unroll
        for (int i = 0; i < T::BLD; ++i)
          rb[i] = Bc[(int64_t)(b_kk + i * T::BROWS) * p.ldb + b_col];
      } else {
#pragma unroll
        for (int i = 0; i < T::ALD; ++i) {
          const int row = a_row + i * T::AROWS;
          ra[i] = (row < it.h && a_kk < clen) ? Ac[(int64_t)row * p.lda + a_kk] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < T::BLD; ++i) {
          const int kk = b_kk + i * T::BROWS;
          rb[i] = (b_col < it.w && kk < clen) ? Bc[(int64_t)kk * p.ldb + b_col] : 0.0;
        }
      }
    };
    auto store_chunk = [&](double* As) {
      double* Bs = As + T::AS;
#pragma unroll
      for (int i = 0; i < T::ALD; ++i) As[(a_row + i * T::AROWS) * T::ASTR + a_kk] = ra[i];
#pragma unroll
      for (int i = 0; i < T::BLD; ++i) Bs[(b_kk + i * T::BROWS) * T::BSTR + b_col] = rb[i];
    };

    // Chunk [c0, c0 + clen) lies inside the inner step ending at s_end.
    int c0 = k0;
    int s_end = min(k0 + bstep, k1);
    bool have = c0 < k1;
    if (have) {
      load_chunk(c0, min(KC, s_end - c0));
      store_chunk(smem);
    }
    __syncthreads();
    int buf = 0;
    while (have) {
      // next chunk: continue in this inner step, or start the next one
      int n0 = c0 + KC, n_end = s_end;
      if (n0 >= s_end) {
        n0 = s_end;
        n_end = min(s_end + bstep, k1);
      }
      const bool have_next = n0 < k1;
      if (have_next) load_chunk(n0, min(KC, n_end - n0));

      const double* As = smem + buf * (T::AS + T::BS);
      const double* Bs = As + T::AS;
      const double* Aw = As + (wm * T::WTM + l16) * T::ASTR + lq;
      const double* Bw = Bs + lq * T::BSTR + wn * T::WTN + l16;
#pragma unroll
      for (int q = 0; q < KC / 4; ++q) {
        double af[T::FM], bf[T::FN];
#pragma unroll
        for (int fm = 0; fm < T::FM; ++fm) af[fm] = Aw[fm * 16 * T::ASTR + q * 4];
#pragma unroll
        for (int fn = 0; fn < T::FN; ++fn) bf[fn] = Bw[q * 4 * T::BSTR + fn * 16];
#pragma unroll
        for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
          for (int fn = 0; fn < T::FN; ++fn)
            acc[fm][fn] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[fm], bf[fn], acc[fm][fn], 0, 0, 0);
      }
      if (have_next) store_chunk(smem + (buf ^ 1) * (T::AS + T::BS));
      __syncthreads();
      buf ^= 1;
      c0 = n0;
      s_end = n_end;
      have = have_next;
    }

    // ---- store C ------------------------------------------------------------
#pragma unroll
    for (int fm = 0; fm < T::FM; ++fm) {
#pragma unroll
      for (int fn = 0; fn < T::FN; ++fn) {
        const int col = wn * T::WTN + fn * 16 + l16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = wm * T::WTM + fm * 16 + 4 * v + lq;
          if (full_tile || (row < it.h && col < it.w))
            Cb[(int64_t)row * p.ldc + col] = acc[fm][fn][v];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Direct-to-LDS variant (buffer_load_dwordx4 ... lds): the chunk loads go
// from global memory straight into an NS-stage LDS ring, with no staging
// registers, so several chunks are in flight per workgroup.  Each
// wave-instruction writes 64 consecutive 16-byte LDS units; which global
// 16 bytes each lane fetches is free, so the ring holds swizzled images:
//   A stage: As[row][u'] (row = 128 B = 8 units of 2 doubles),
//            u' = u ^ ((row / 2) % 8)     -> fragment reads conflict-free
//   B stage: Bs[k][u'] (row = TN doubles), u' = u ^ (8 (k % 2))
// The loads go through buffer descriptors rebased at every chunk (A at the
// item's first row and the chunk's first column, B at the chunk's first row
// and the item's first column), so each lane keeps one 32-bit byte offset
// per instruction for the whole item.  Lanes whose source is outside the
// item (ragged rows/cols, or k past a short chunk) take an offset past the
// descriptor's range, which the hardware returns as zeros.  Used when every
// 16-byte unit is either wholly inside or wholly outside the k-range (even k
// bounds, even leading dimensions, even column offsets, 16-byte aligned
// operands) and the offsets fit in 31 bits; otherwise the staged kernel
// above runs.
constexpr uint32_t kDmaOut = 0x80000000u;   // descriptor range; offsets >= it read zero

template <int TM, int TN, int NS, int WM, int WN, int OCC>
__global__ __launch_bounds__(WM * WN * 64, OCC)
void fp64_dma_kernel(UpdateArgs p) {
  constexpr int KC = 16;
  constexpr int NT = WM * WN * 64, NW = WM * WN;
  constexpr int WTM = TM / WM, WTN = TN / WN, FM = WTM / 16, FN = WTN / 16;
  constexpr int ABYTES = TM * KC * 8, BBYTES = KC * TN * 8, SBYTES = ABYTES + BBYTES;
  constexpr int AINS = ABYTES / 1024 / NW;   // A wave-instructions per wave per chunk
  constexpr int BINS = BBYTES / 1024 / NW;
  constexpr int BUPR = TN / 2;               // 16-byte units per B row
  static_assert(ABYTES % (1024 * NW) == 0 && BBYTES % (1024 * NW) == 0, "load split");
  static_assert(TN % 16 == 0 && BUPR >= 16, "B swizzle needs >= 16 units per row");
  __shared__ __attribute__((aligned(1024))) uint8_t smem[NS * SBYTES];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: LDS targets in SGPRs
  const int wm = wave / WN, wn = wave % WN;
  const int l16 = lane & 15, lq = lane >> 4;
  const int k0 = (int)p.k0, k1 = (int)p.k1, bstep = (int)p.bstep;
  if (p.gate && *p.gate != 0) return;

  const int bid = blockIdx.x, xcd = bid & 7, slot0 = bid >> 3;
  const int slots = p.persistent ? (gridDim.x + 7 - xcd) >> 3 : 1;

  for (int slot = slot0;; slot += slots) {
    if (!p.persistent && slot != slot0) break;
    if (slot >= p.per_xcd) break;
    const int idx = xcd * p.per_xcd + slot;
    if (idx >= p.nitems) break;
    const WorkItem it = fetch_item<TM, TN>(p, idx);
    const bool full_tile = (it.h == TM) && (it.w == TN);
    const double* Ab = p.A + (int64_t)it.r0 * p.lda;
    const double* Bb = p.B + it.c0;
    double* Cb = p.C + (int64_t)it.r0 * p.ldc + it.c0;

    // Per-item byte offsets of this wave's DMA units from the chunk's
    // buffer bases (kDmaOut for units outside the item).
    uint32_t aoff[AINS], boff[BINS];
    int bkk[BINS], au2[AINS];
#pragma unroll
    for (int j = 0; j < AINS; ++j) {
      const int t = wave * AINS + j;               // 1 KB block: rows 8t .. 8t+7
      const int row = 8 * t + (lane >> 3);
      const int u = (lane & 7) ^ ((row >> 1) & 7);
      au2[j] = 2 * u;
      aoff[j] = row < it.h ? (uint32_t)((int64_t)row * p.lda * 8 + 16 * u) : kDmaOut;
    }
#pragma unroll
    for (int j = 0; j < BINS; ++j) {
      const int t = wave * BINS + j;               // 1 KB block of B rows
      const int unit = t * 64 + lane;              // LDS unit in the stage
      const int kk = unit / BUPR, us = unit % BUPR;
      const int u = us ^ (8 * (kk & 1));
      bkk[j] = kk;
      boff[j] = 2 * u < it.w ? (uint32_t)((int64_t)kk * p.ldb * 8 + 16 * u) : kDmaOut;
    }
    // issue the DMA loads of chunk [c0, c0 + clen) into ring stage `st`
    auto issue = [&](int c0, int clen, int st) {
      uint8_t* sA = smem + st * SBYTES;
      uint8_t* sB = sA + ABYTES;
      const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
          (void*)(Ab + c0), (short)0, (int)kDmaOut, kBufferWord3);
      const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
          (void*)(Bb + (int64_t)c0 * p.ldb), (short)0, (int)kDmaOut, kBufferWord3);
      // a short chunk (a step's ragged end) also zeroes the units past clen
      auto put = [&](auto shortc) {
#pragma unroll
        for (int j = 0; j < AINS; ++j) {
          const uint32_t off = shortc && au2[j] >= clen ? kDmaOut : aoff[j];
          __builtin_amdgcn_raw_ptr_buffer_load_lds(
              ra, (__attribute__((address_space(3))) void*)(sA + (wave * AINS + j) * 1024), 16,
              off, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < BINS; ++j) {
          const uint32_t off = shortc && bkk[j] >= clen ? kDmaOut : boff[j];
          __builtin_amdgcn_raw_ptr_buffer_load_lds(
              rb, (__attribute__((address_space(3))) void*)(sB + (wave * BINS + j) * 1024), 16,
              off, 0, 0, 0);
        }
      };
      if (clen < KC) put(std::true_type{});
      else put(std::false_type{});
    };

    d4 acc[FM][FN];
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < FN; ++fn)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[fm][fn][v] = 0.0;
    // C first: its loads are then older than every chunk load of the item.
    // Addresses are clamped into the item so that every load is
    // unconditional (measured 1.5 % faster than predicated loads); values
    // loaded for lanes outside the item are never stored.
    if (!p.zero_init) {
#pragma unroll
      for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) {
          const int col = min(wn * WTN + fn * 16 + l16, it.w - 1);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = min(wm * WTM + fm * 16 + 4 * v + lq, it.h - 1);
            acc[fm][fn][v] = Cb[(int64_t)row * p.ldc + col];
          }
        }
    }

    // chunk schedule (inner steps of bstep from k0, KC-chunks inside each)
    int q_c0 = k0, q_end = min(k0 + bstep, k1);  // next chunk to issue
    auto next_chunk = [&](int& c0, int& clen) {
      c0 = q_c0;
      clen = min(KC, q_end - q_c0);
      int n0 = q_c0 + KC;
      if (n0 >= q_end) {
        n0 = q_end;
        q_end = min(q_end + bstep, k1);
      }
      q_c0 = n0;
    };
    int nchunks = 0;
    for (int s0 = k0; s0 < k1; s0 += bstep) nchunks += (min(s0 + bstep, k1) - s0 + KC - 1) / KC;
    // prologue: NS - 1 chunks in flight
#pragma unroll
    for (int st = 0; st < NS - 1; ++st) {
      if (st < nchunks) {
        int c0, clen;
        next_chunk(c0, clen);
        issue(c0, clen, st);
      }
    }
    for (int ci = 0; ci < nchunks; ++ci) {
      // chunk ci's own loads must be complete; the ones issued after it may
      // stay in flight (vmcnt counts this wave's loads in issue order)
      const int ahead = min(NS - 2, nchunks - 1 - ci);
      if (NS >= 4 && ahead >= 2)
        asm volatile("s_waitcnt vmcnt(%0)" ::"n"(2 * (AINS + BINS)) : "memory");
      else if (NS >= 3 && ahead >= 1)
        asm volatile("s_waitcnt vmcnt(%0)" ::"n"(AINS + BINS) : "memory");
      else
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      ring_barrier();
      // refill the stage consumed in the previous iteration
      if (ci + NS - 1 < nchunks) {
        int c0, clen;
        next_chunk(c0, clen);
        issue(c0, clen, (ci + NS - 1) % NS);
      }
      const uint8_t* sA = smem + (ci % NS) * SBYTES;
      const uint8_t* sB = sA + ABYTES;
      // raised priority while this wave feeds the matrix core, so the other
      // workgroup's waves on the SIMD issue their loads and barrier work in
      // its gaps (measured 0.6 % faster)
      __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int q = 0; q < KC / 4; ++q) {
        double af[FM], bf[FN];
        const int k = 4 * q + lq;
#pragma unroll
        for (int fm = 0; fm < FM; ++fm) {
          const int row = wm * WTM + fm * 16 + l16;
          const int u = (k >> 1) ^ ((row >> 1) & 7);
          af[fm] = *(const double*)(sA + row * 128 + u * 16 + (k & 1) * 8);
        }
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) {
          const int col = wn * WTN + fn * 16 + l16;
          const int u = (col >> 1) ^ (8 * (k & 1));
          bf[fn] = *(const double*)(sB + k * TN * 8 + u * 16 + (col & 1) * 8);
        }
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
          for (int fn = 0; fn < FN; ++fn)
            acc[fm][fn] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[fm], bf[fn], acc[fm][fn], 0, 0, 0);
      }
      __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();  // the ring is reused by the next item

#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < FN; ++fn) {
        const int col = wn * WTN + fn * 16 + l16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = wm * WTM + fm * 16 + 4 * v + lq;
          if (full_tile || (row < it.h && col < it.w))
            Cb[(int64_t)row * p.ldc + col] = acc[fm][fn][v];
        }
      }
  }
}

namespace {
struct Fp64Entry {
  TileCfg cfg;
  void (*kern)(UpdateArgs);
  int threads;
  int occupancy;
};

#define HS_FP64(TM, TN, KC, WM, WN, OCC)                                                 \
  Fp64Entry{TileCfg{TM, TN, KC, WM * WN}, fp64_update_kernel<TM, TN, KC, WM, WN, OCC>,    \
            WM * WN * 64, OCC}

const std::vector<Fp64Entry>& table() {
  static const std::vector<Fp64Entry> t = {
      HS_FP64(128, 128, 16, 2, 2, 2),
      HS_FP64(128, 128, 8, 2, 2, 2),
      HS_FP64(256, 128, 8, 4, 2, 1),
      HS_FP64(256, 128, 16, 4, 2, 1),
      HS_FP64(128, 64, 8, 2, 2, 2),
      HS_FP64(128, 128, 32, 2, 2, 1),
      HS_FP64(128, 64, 16, 2, 2, 2),
      HS_FP64(64, 128, 16, 2, 2, 2),
      HS_FP64(64, 64, 16, 2, 2, 4),
      HS_FP64(64, 64, 32, 2, 2, 2),
      HS_FP64(32, 32, 16, 2, 2, 8),
      // wider tiles and another wave count (tuner candidates).  No 256 x 256:
      // its FP64 accumulators alone (512 KB) are a CU's whole register file.
      HS_FP64(128, 256, 16, 2, 4, 1),
      HS_FP64(64, 256, 16, 1, 4, 1),
      HS_FP64(256, 64, 16, 4, 1, 1),
      HS_FP64(128, 128, 16, 4, 2, 1),
  };
  return t;
}

struct DmaEntry {
  TileCfg cfg;
  void (*kern)(UpdateArgs);
  int threads;
  int occupancy;
};
#define HS_DMA(TM, TN, NS, WM, WN, OCC)                                                  \
  DmaEntry{TileCfg{TM, TN, 16, WM * WN}, fp64_dma_kernel<TM, TN, NS, WM, WN, OCC>,        \
           WM * WN * 64, OCC}
// direct-to-LDS kernels, keyed by the staged kernel configuration they replace
const std::vector<DmaEntry>& dma_table() {
  static const std::vector<DmaEntry> t = {
      HS_DMA(128, 128, 2, 2, 2, 2),
      HS_DMA(256, 128, 3, 4, 2, 1),
      HS_DMA(64, 64, 4, 2, 2, 2),
      HS_DMA(128, 64, 3, 2, 2, 2),
      HS_DMA(64, 128, 3, 2, 2, 2),
      HS_DMA(128, 256, 2, 2, 4, 1),
      HS_DMA(64, 256, 3, 1, 4, 1),
      HS_DMA(256, 64, 3, 4, 1, 1),
      HS_DMA(128, 128, 3, 4, 2, 1),
  };
  return t;
}
}  // namespace

const std::vector<TileCfg>& fp64_configs() {
  static std::vector<TileCfg> c = [] {
    std::vector<TileCfg> v;
    for (auto& e : table()) v.push_back(e.cfg);
    return v;
  }();
  return c;
}

int fp64_occupancy(const TileCfg& cfg) {
  for (auto& e : table())
    if (same_tile(cfg, e.cfg)) return e.occupancy;
  return 0;
}

bool fp64_has_dma(const TileCfg& cfg) {
  for (auto& e : dma_table())
    if (same_tile(cfg, e.cfg)) return true;
  return false;
}

hipError_t launch_fp64_dense(const double* A, int64_t lda, const double* B, int64_t ldb,
                             double* C, int64_t ldc, int64_t m, int64_t n, int64_t k,
                             hipStream_t s, int64_t m2, int64_t n2) {
  if (m2 <= 0 || n2 <= 0) m2 = n2 = 0;
  if (m <= 0 || n <= 0) {
    if (!m2) return hipSuccess;
    // only the second block: it is then the first, shifted by n columns
    return launch_fp64_dense(A, lda, B + n, ldb, C + n, ldc, m2, n2, k, s);
  }
  const bool small = m < 512 || n < 512 || (m2 && (m2 < 512 || n2 < 512));
  const TileCfg cfg = small ? TileCfg{64, 64, 16} : TileCfg{128, 128, 16};
  UpdateArgs a{};
  a.A = A; a.lda = lda; a.B = B; a.ldb = ldb; a.C = C; a.ldc = ldc;
  a.items = nullptr;
  a.dense_m = (int32_t)m; a.dense_n = (int32_t)n;
  a.dense_nc = (int32_t)((n + cfg.tn - 1) / cfg.tn);
  a.dense_items1 = (int32_t)((m + cfg.tm - 1) / cfg.tm) * a.dense_nc;
  a.dense_m2 = (int32_t)m2; a.dense_n2 = (int32_t)n2;
  a.dense_nc2 = (int32_t)((n2 + cfg.tn - 1) / cfg.tn);
  const int64_t nit = (int64_t)a.dense_items1 + (int64_t)((m2 + cfg.tm - 1) / cfg.tm) * a.dense_nc2;
  a.nitems = (int32_t)nit;
  a.per_xcd = (int32_t)((nit + 7) / 8);
  a.k0 = 0; a.k1 = k; a.bstep = k; a.zero_init = 0; a.persistent = 0; a.gate = nullptr;
  // 16-byte DMA units: even k, leading dimensions, column offsets and widths
  const bool dma = !((k | lda | ldb) & 1) && !(((uintptr_t)A | (uintptr_t)B) & 15) &&
                   (int64_t)cfg.tm * lda * 8 < (int64_t(1) << 31) &&
                   (int64_t)16 * ldb * 8 < (int64_t(1) << 31) && !(n & 1) && !(n2 & 1);
  return launch_fp64(cfg, a, 8 * a.per_xcd, s, dma);
}

hipError_t launch_fp64(const TileCfg& cfg, const UpdateArgs& a, int grid, hipStream_t s,
                       bool dma) {
  if (dma) {
    for (auto& e : dma_table()) {
      if (same_tile(cfg, e.cfg)) {
        hipLaunchKernelGGL(e.kern, dim3(grid), dim3(e.threads), 0, s, a);
        return hipGetLastError();
      }
    }
  }
  for (auto& e : table()) {
    if (same_tile(cfg, e.cfg)) {
      hipLaunchKernelGGL(e.kern, dim3(grid), dim3(e.threads), 0, s, a);
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace hs
