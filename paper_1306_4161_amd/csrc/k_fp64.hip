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

  const int bid = blockIdx.x;
  const int xcd = bid & 7;
  const int slot0 = bid >> 3;
  const int slots = p.persistent ? (gridDim.x + 7 - xcd) >> 3 : 1;

  for (int slot = slot0;; slot += slots) {
    if (!p.persistent && slot != slot0) break;
    if (slot >= p.per_xcd) break;
    const int idx = xcd * p.per_xcd + slot;
    if (idx >= p.nitems) break;
    const WorkItem it = p.items[idx];
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

namespace {
struct Fp64Entry {
  TileCfg cfg;
  void (*kern)(UpdateArgs);
  int threads;
  int occupancy;
};

#define HS_FP64(TM, TN, KC, WM, WN, OCC) \
  Fp64Entry{TileCfg{TM, TN, KC}, fp64_update_kernel<TM, TN, KC, WM, WN, OCC>, WM * WN * 64, OCC}

const std::vector<Fp64Entry>& table() {
  static const std::vector<Fp64Entry> t = {
      HS_FP64(128, 128, 16, 2, 2, 2),
      HS_FP64(128, 128, 8, 2, 2, 2),
      HS_FP64(256, 128, 8, 4, 2, 1),
      HS_FP64(128, 64, 8, 2, 2, 2),
      HS_FP64(128, 128, 32, 2, 2, 1),
      HS_FP64(128, 64, 16, 2, 2, 2),
      HS_FP64(64, 128, 16, 2, 2, 2),
      HS_FP64(64, 64, 16, 2, 2, 4),
      HS_FP64(64, 64, 32, 2, 2, 2),
      HS_FP64(32, 32, 16, 2, 2, 8),
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
    if (e.cfg.tm == cfg.tm && e.cfg.tn == cfg.tn && e.cfg.kc == cfg.kc) return e.occupancy;
  return 0;
}

hipError_t launch_fp64(const TileCfg& cfg, const UpdateArgs& a, int grid, hipStream_t s) {
  for (auto& e : table()) {
    if (e.cfg.tm == cfg.tm && e.cfg.tn == cfg.tn && e.cfg.kc == cfg.kc) {
      hipLaunchKernelGGL(e.kern, dim3(grid), dim3(e.threads), 0, s, a);
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace hs
