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
// MFMA operand layout (16x16x4, FP64, wave64):
//   A fragment: lane l holds A[l % 16][l / 16]  (16 x 4 block)
//   B fragment: lane l holds B[l / 16][l % 16]  (4 x 16 block)
//   D:          lane l, item v holds D[4 * v + l / 16][l % 16]
//
// LDS layouts (doubles):
//   As[row][k] with row stride KC + 1: the 16 rows x 4 k of an A fragment
//      fall on distinct banks.
//   Bs[k][col] with row stride TN + 16: the 4 k-rows of a B fragment are
//      half a bank-cycle apart.
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
  static_assert(TM % (WM * 16) == 0 && TN % (WN * 16) == 0, "wave tiling");
  static_assert((TM * KC) % NT == 0 && (TN * KC) % NT == 0, "load tiling");
  static_assert(KC % 4 == 0, "chunk is whole MFMA k-groups");
};

template <int TM, int TN, int KC, int WM, int WN>
__global__ __launch_bounds__(WM * WN * 64)
void fp64_update_kernel(UpdateArgs p) {
  using T = Fp64Tile<TM, TN, KC, WM, WN>;
  __shared__ double smem[2 * (T::AS + T::BS)];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int l16 = lane & 15, lq = lane >> 4;

  // Chunk schedule of the launch: inner steps of length bstep from k0.
  const int64_t klen = p.k1 - p.k0;
  const int64_t nsteps = (klen + p.bstep - 1) / p.bstep;
  const int64_t cps = (p.bstep + KC - 1) / KC;              // chunks per full step
  const int64_t last_len = klen - (nsteps - 1) * p.bstep;
  const int64_t nchunks = (nsteps - 1) * cps + (last_len + KC - 1) / KC;

  // Work items: in the plain launch one per workgroup, placed so that the
  // items of one XCD-list are contiguous (workgroup w runs on XCD w % 8);
  // in persistent mode each workgroup strides through its XCD's list.
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

    d4 acc[T::FM][T::FN];
    // ---- load C (or start from zero) --------------------------------------
#pragma unroll
    for (int fm = 0; fm < T::FM; ++fm) {
#pragma unroll
      for (int fn = 0; fn < T::FN; ++fn) {
        const int col = wn * T::WTN + fn * 16 + l16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = wm * T::WTM + fm * 16 + 4 * v + lq;
          double c = 0.0;
          if (!p.zero_init && row < it.h && col < it.w)
            c = p.C[(int64_t)(it.r0 + row) * p.ldc + it.c0 + col];
          acc[fm][fn][v] = c;
        }
      }
    }

    double ra[T::ALD], rb[T::BLD];
    auto chunk_range = [&](int64_t ci, int64_t& c0, int64_t& cend) {
      const int64_t st = ci / cps;
      const int64_t s0 = p.k0 + st * p.bstep;
      const int64_t s1 = min(s0 + p.bstep, p.k1);
      c0 = s0 + (ci - st * cps) * KC;
      cend = min(c0 + (int64_t)KC, s1);
    };
    auto load_chunk = [&](int64_t ci) {
      int64_t c0, cend;
      chunk_range(ci, c0, cend);
#pragma unroll
      for (int i = 0; i < T::ALD; ++i) {
        const int e = tid + i * T::NT;
        const int row = e / KC, kk = e % KC;
        double v = 0.0;
        if (row < it.h && c0 + kk < cend)
          v = p.A[(int64_t)(it.r0 + row) * p.lda + c0 + kk];
        ra[i] = v;
      }
#pragma unroll
      for (int i = 0; i < T::BLD; ++i) {
        const int e = tid + i * T::NT;
        const int kk = e / TN, col = e % TN;
        double v = 0.0;
        if (col < it.w && c0 + kk < cend)
          v = p.B[(c0 + kk) * p.ldb + it.c0 + col];
        rb[i] = v;
      }
    };
    auto store_chunk = [&](int buf) {
      double* As = smem + buf * (T::AS + T::BS);
      double* Bs = As + T::AS;
#pragma unroll
      for (int i = 0; i < T::ALD; ++i) {
        const int e = tid + i * T::NT;
        As[(e / KC) * T::ASTR + e % KC] = ra[i];
      }
#pragma unroll
      for (int i = 0; i < T::BLD; ++i) {
        const int e = tid + i * T::NT;
        Bs[(e / TN) * T::BSTR + e % TN] = rb[i];
      }
    };

    if (nchunks > 0) {
      load_chunk(0);
      store_chunk(0);
    }
    __syncthreads();
    for (int64_t ci = 0; ci < nchunks; ++ci) {
      const int buf = (int)(ci & 1);
      if (ci + 1 < nchunks) load_chunk(ci + 1);
      const double* As = smem + buf * (T::AS + T::BS);
      const double* Bs = As + T::AS;
#pragma unroll
      for (int q = 0; q < KC / 4; ++q) {
        double af[T::FM], bf[T::FN];
#pragma unroll
        for (int fm = 0; fm < T::FM; ++fm)
          af[fm] = As[(wm * T::WTM + fm * 16 + l16) * T::ASTR + q * 4 + lq];
#pragma unroll
        for (int fn = 0; fn < T::FN; ++fn)
          bf[fn] = Bs[(q * 4 + lq) * T::BSTR + wn * T::WTN + fn * 16 + l16];
#pragma unroll
        for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
          for (int fn = 0; fn < T::FN; ++fn)
            acc[fm][fn] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[fm], bf[fn], acc[fm][fn], 0, 0, 0);
      }
      if (ci + 1 < nchunks) store_chunk(buf ^ 1);
      __syncthreads();
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
          if (row < it.h && col < it.w)
            p.C[(int64_t)(it.r0 + row) * p.ldc + it.c0 + col] = acc[fm][fn][v];
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
  Fp64Entry{TileCfg{TM, TN, KC}, fp64_update_kernel<TM, TN, KC, WM, WN>, WM * WN * 64, OCC}

const std::vector<Fp64Entry>& table() {
  static const std::vector<Fp64Entry> t = {
      HS_FP64(128, 128, 16, 2, 2, 2),
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
