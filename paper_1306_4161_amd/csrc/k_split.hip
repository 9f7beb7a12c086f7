// Precision form of the local update: FP64 operands split into small-integer
// digit planes (BF16, FP8-e4m3 or INT8), products of the planes on the matrix
// cores with FP32 (INT32) accumulation that is exact by construction, and
// FP64 recombination.  An error-free splitting in the spirit of Ozaki, Ogita,
// Oishi and Rump (Numer. Algorithms 59, 2012); not part of the HSUMMA paper,
// which only fixes the update C += A_panel x B_panel being computed.
//
// Digit rule, per outer panel (k-columns [k0, k0 + w)):
//   e_i  = smallest integer with max_l |a_il| <= 2^e_i   (A row i; 0 if zero)
//   f_j  = the same over B column j
//   x    = a 2^-e in [-1, 1];  d_1 = rint(x 2^H), r_1 = x 2^H - d_1,
//          d_l = rint(r_{l-1} 2^T), r_l = r_{l-1} 2^T - d_l   (round half even)
//   BF16: H = 8, T = 9; FP8-e4m3: H = 4, T = 5; every |d| <= 2^H, exact in
//   the narrow format.  INT8: H = 6, T = 8 (digits in [-64, 64] and
//   [-128, 128]), then a carry pass from the last of the s digits to the
//   second turns a digit of 128 (129 after a carry) into itself minus 256
//   with one added to the digit before it: same value, every later digit in
//   [-128, 127], the first in [-64, 65].  BF16 planes hold d_l 2^(-T (l-1)) (a power-of-two
//   scale, still exact) so that the product of planes l1 and l2 already
//   carries its weight 2^(-T (l1 + l2 - 2)).
//
// Products: the digit pairs (l1, l2) with l1 + l2 <= s + 1 (1-based), s the
// panel's slice count.  Pairs of one level L = l1 + l2 share an FP32
// accumulator.  BF16: levels 2..5 are exact accumulators (at most 4 pairs
// x 64 k x 2^16 <= 2^24), deeper levels (weight <= 2^-36) share one
// accumulator whose FP32 rounding stays below 2^-60 of the leading term;
// each accumulator is added into an FP64 panel sum within its exactness
// bound (every 64 or 128 k).  FP8: every
// level is exact over the whole panel (7 pairs x 2^8 x w <= 2^24 for
// w <= 9362) and is added, scaled by 2^(-T (L - 2)), at the end of the panel.
// INT8: every level is exact in INT32 over the whole panel (8 pairs x 2^14 x
// w < 2^31 for w <= 8192) and is added the same way.
// Finally C += 2^(e_i + f_j - 2H) x panel sum, in FP64.
#include <type_traits>

#include "internal.h"
#include "split.h"

namespace hs {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef int i4v __attribute__((ext_vector_type(4)));
typedef int i16v __attribute__((ext_vector_type(16)));

// Compile-time loop: f(std::integral_constant<int, I>) for I = B .. E-1.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// digit format FMT (0: BF16, 1: FP8-e4m3, 2: INT8): first shift H, later
// shift T, bytes per stored digit
constexpr int digit_h(int fmt) { return fmt == 0 ? 8 : fmt == 1 ? 4 : 6; }
constexpr int digit_t(int fmt) { return fmt == 0 ? 9 : fmt == 1 ? 5 : 8; }
constexpr int digit_bytes(int fmt) { return fmt == 0 ? 2 : 1; }

// INT8 digits of the 16 values r[] (already scaled by 2^-e): S digits per
// value (round half to even), then the carry pass into the int8 range;
// plane l's 16 bytes are packed into w[l][0..3].  S is a template parameter
// so that the unrolled loops carry no branches.
template <int S>
__device__ __forceinline__ void int8_digits(const double* r, uint32_t (&w)[kSplitMaxSlices][4]) {
  constexpr int s = S;
#pragma unroll
  for (int l = 0; l < kSplitMaxSlices; ++l)
#pragma unroll
    for (int j = 0; j < 4; ++j) w[l][j] = 0u;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    int c[kSplitMaxSlices];
    double x = r[q];
    int shift = digit_h(2);
#pragma unroll
    for (int l = 0; l < kSplitMaxSlices; ++l) {
      c[l] = 0;
      if (l < s) {
        const double y = ldexp(x, shift);
        const double d = rint(y);
        x = y - d;
        c[l] = (int)d;
        shift = digit_t(2);
      }
    }
#pragma unroll
    for (int l = kSplitMaxSlices - 1; l >= 1; --l)
      if (l < s && c[l] >= 128) {
        c[l] -= 256;
        c[l - 1] += 1;
      }
#pragma unroll
    for (int l = 0; l < kSplitMaxSlices; ++l)
      w[l][q >> 2] |= (uint32_t)(uint8_t)(int8_t)c[l] << (8 * (q & 3));
  }
}

__device__ inline int exponent_bound(double mx) {
  if (!(mx > 0.0)) return 0;
  int e;
  const double f = frexp(mx, &e);  // mx = f 2^e, f in [0.5, 1)
  return f == 0.5 ? e - 1 : e;
}

__device__ inline uint8_t e4m3_of_int(int d) {
  // OCP e4m3fn encoding of an integer with |d| <= 16 (exact).
  const int a = d < 0 ? -d : d;
  uint8_t bits = 0;
  if (a) {
    const int E = 31 - __clz(a);          // 0..4
    const int Mt = ((a << 3) >> E) - 8;   // 3-bit mantissa, exact for |d| <= 16
    bits = (uint8_t)(((E + 7) << 3) | Mt);
  }
  return (uint8_t)(bits | (d < 0 ? 0x80 : 0));
}

// Digit planes are stored in k-blocks of the product kernel's step: BF16 and
// FP8 k16-block-major, element (plane, row, kk) at plane * plane_stride +
// (kk / 16) * rows * 16 + row * 16 + kk % 16; INT8 k32-block-major, at
// plane * plane_stride + (kk / 32) * rows * 32 + row * 32 + kk % 32.  So the
// k of one row in one step are contiguous and one step of a plane (all rows)
// is one contiguous run, the unit the product kernel streams.  INT8 digits
// are stored as their two's-complement bytes.

// Slice count of a panel from its statistics.  ka, kb: log2 of the largest
// kappa = max|x| w / sum|x| over the panel's A rows and B columns.  Model of
// the max scaled error of the truncated s-slice product, fitted to the CPU
// oracle at n = 16384 on uniform and exponent-spread (sigma = 2) entries:
// log2 err ~ -bits(s) + 0.75 (ka + kb) + 1 - c, bits(s) = H + T (s - 1).
// The credit c = log2(k) / 2 holds when the truncation errors of the k terms
// of an entry add with random signs while (|A||B|)_ij grows like k; it is
// given only when no line's low-order bits repeat: ca, cb are the largest
// |sum r| / sum |r| over the lines, r the part of each |x| below its 41st
// significant bit, about 1.2 / sqrt(w) for varied values and 1 for lines
// of repeated magnitudes (whose dropped digit products then add up
// coherently).  The smallest s whose estimate is within 2^-tau is taken.
// kappa cannot exceed the panel width w, so when ka or kb comes within 1.5
// bits of log2 w (the largest element is over a third of its line's sum) the
// statistic no longer measures the spread (narrow panels, or lines dominated
// by one element) and the estimate is only a lower bound.
// Such a panel takes smax unless the geometric spread says otherwise: la, lb
// are the largest log2 max|x| - mean log2|x| over the lines (which does not
// saturate), and the second estimate log2 err ~ -bits(s) + 0.66 (la + lb) +
// 7.73 - 1.11 log2 k is fitted, like the first, to the CPU oracle's
// truncated products (exponent spreads sigma = 2 ... 4, k = 64 ... 16384,
// saturated panels only; largest residual 2.6 bits, hence one bit of margin
// on top of tau).  If either estimate needs more than smax slices the panel
// goes to the FP64 kernel.
// BF16 levels beyond the fourth share one FP32 accumulator that rounds: its
// error, of the order of 2^-60.5 kappa_A kappa_B / sqrt(k) of (|A||B|)_ij
// (measured up to 9 times that at sigma = 3, k = 1024, 7 digits), is above
// the truncation error of the largest count, so a BF16 panel whose estimate
// needs more than kBf16RoundBits bits also goes to the FP64 kernel (measured:
// sigma = 2.5 and 3 panels the truncation model accepts at 7 digits reach
// 4-6e-14 on the GPU, and 9e-15 two panels outside the saturated band
// whose estimate was 56.05 bits).
// Returns 0 -- the panel goes to the FP64 kernel -- when the panel holds a
// non-finite value (whose IEEE propagation the digits cannot carry) or when
// the estimate needs more than smax slices.  A fixed count is used as given
// (non-finite panels still go to the FP64 kernel).
// The digit pass evaluates it once per panel and stores the result, which
// the product kernels and the FP64 route read.
constexpr float kBf16RoundBits = 56.0f;

__device__ __forceinline__ int panel_slices(const uint32_t* stats, int fixed_s, int smin, int smax,
                                            int tau_bits, float log2k, float log2w, int H, int T) {
  // BF16 is the format with H = 8, T = 9
  const float cap = (H == 8 && T == 9) ? kBf16RoundBits : 1e30f;
  if (stats[kStatNonFinite]) return 0;
  if (fixed_s > 0) return min(kSplitMaxSlices, fixed_s);
  const int top = min(smax, kSplitMaxSlices);
  const float ka = __uint_as_float(stats[kStatKappaA]), kb = __uint_as_float(stats[kStatKappaB]);
  const float coh = fmaxf(__uint_as_float(stats[kStatCohA]), __uint_as_float(stats[kStatCohB]));
  const bool cancels = log2w >= 6.0f && coh <= fminf(0.75f, 8.0f * exp2f(-0.5f * log2w));
  const float need =
      (float)tau_bits + 0.75f * (ka + kb) + 1.0f - (cancels ? 0.5f * log2k : 0.0f);
  const int s = max(smin, (int)ceilf((need - (float)H) / (float)T) + 1);
  if (s > top || need > cap) return 0;
  if (fmaxf(ka, kb) >= log2w - 1.5f) {
    const float lam = __uint_as_float(stats[kStatLamA]) + __uint_as_float(stats[kStatLamB]);
    const float need2 =
        (float)tau_bits + 0.66f * lam + 8.73f - (cancels ? 1.11f * log2k : 0.0f);
    if ((int)ceilf((need2 - (float)H) / (float)T) + 1 > top || need2 > cap) return 0;
    return max(1, top);
  }
  return max(1, s);
}

// log2 |x| for finite nonzero x, from its exponent and mantissa (no underflow
// to the FP32 range).
__device__ __forceinline__ float log2_abs(double x) {
  int e;
  const double m = frexp(fabs(x), &e);               // [0.5, 1)
  return (float)e + __log2f((float)m);
}

// The bits of |x| below its 41st significant bit, as a signed fraction of
// that bit's unit in [-1/2, 1/2] (0 for 0 and for non-finite x): repeated
// magnitudes give equal values, varied ones values spread over the interval.
__device__ __forceinline__ double low_bits(double x) {
  if (!(fabs(x) <= 1.7976931348623157e308)) return 0.0;
  int e;
  const double y = ldexp(frexp(fabs(x), &e), 41);   // exact: mantissa times 2^41
  return y - rint(y);
}

// The panel's coherence statistic from one line's sums.
__device__ __forceinline__ float coherence(double rs, double ra) {
  return ra > 0.0 ? (float)(fabs(rs) / ra) : 0.0f;
}

// ---- split: statistics, their combination, digits ---------------------------
// A line is a row of A or a column of B (line index: A rows 0 .. m-1, then
// B columns m .. m+n-1).  The panel is cut into blocks of 64 lines x one
// 64-k slab, 4 waves each: wave w owns the 16-k tile [64 slab + 16 w, + 16),
// one line per lane, with no loop, so that many blocks are in flight per CU
// and narrow problems (few lines, a wide panel) still fill the chip.  A rows
// are staged through a per-wave LDS tile, read as 8 rows x 128 bytes per
// wave-load and then one row per lane (row stride 18 doubles: the 16-byte
// reads of 16 lanes hit distinct banks); B columns are read directly, one
// 512-byte row segment per wave-load.
//   1. statistics: each line's partial sums over the slab (max |x|, sum |x|,
//      the coherence sums, the log-magnitude sum and count) go to the
//      workspace, field-major, slab by slab;
//   2. combination: one thread per line adds its partials in slab order (so
//      the result does not depend on scheduling), writes the line's
//      exponent and folds the line into the panel's statistics;
//   3. digits: the panel's slice count from its statistics, then the digit
//      planes of each tile (only those planes).
constexpr int kSplitWaves = 4;               // waves per block
constexpr int kSlabK = 16 * kSplitWaves;     // k per block
constexpr int kTileStride = 18;              // doubles per staged row
constexpr int kPartFields = 6;               // partial sums per line and slab

// The 64 x 16 tile of A rows [64 blk, + 64) (clamped to the last row) and
// panel columns [k0, k0 + 16) (zero at and past w) into this wave's LDS
// tile, then row `lane` of it into x.
__device__ __forceinline__ void load_row_tile(const SplitArgs& p, int blk, int k0, double* tile,
                                              double (&x)[16]) {
  const int lane = threadIdx.x & 63;
  const int lr = lane >> 3, kp = 2 * (lane & 7);   // load role: row lr + 8 i, k pair kp
  double v[16];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int row = min(blk * 64 + lr + 8 * i, p.m - 1);
    const double* rp = p.A + (int64_t)row * p.lda + p.k0 + k0 + kp;
    v[2 * i] = k0 + kp < p.w ? rp[0] : 0.0;
    v[2 * i + 1] = k0 + kp + 1 < p.w ? rp[1] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    double* t = tile + (lr + 8 * i) * kTileStride + kp;
    t[0] = v[2 * i];
    t[1] = v[2 * i + 1];
  }
  // the same wave reads the tile back: its LDS accesses complete in order
#pragma unroll
  for (int q = 0; q < 16; ++q) x[q] = tile[lane * kTileStride + q];
}

// Panel columns [k0, k0 + 16) of B column `col` (zero at and past w).
__device__ __forceinline__ void load_col_tile(const SplitArgs& p, int col, int k0, double (&x)[16]) {
#pragma unroll
  for (int q = 0; q < 16; ++q)
    x[q] = k0 + q < p.w ? p.B[(int64_t)(p.k0 + k0 + q) * p.ldb + col] : 0.0;
}

__global__ __launch_bounds__(64 * kSplitWaves) void split_stats_kernel(SplitArgs p) {
  // the staging tiles, then (once every wave has read its tile) the waves'
  // partial sums [wave][field][lane]: 37 KB, four blocks per CU
  __shared__ double tiles[kSplitWaves][64 * kTileStride];
  static_assert(kSplitWaves * kPartFields * 64 <= kSplitWaves * 64 * kTileStride, "reuse");
  double* red = &tiles[0][0];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ga = (p.m + 63) / 64;
  const bool rows = (int)blockIdx.x < ga;
  const int blk = rows ? blockIdx.x : blockIdx.x - ga;
  const int nl = rows ? p.m : p.n;
  const int line = blk * 64 + lane;
  const bool valid = line < nl;
  const int k0 = blockIdx.y * kSlabK + 16 * wave;
  double x[16];
  if (rows) load_row_tile(p, blk, k0, tiles[wave], x);
  else load_col_tile(p, valid ? line : nl - 1, k0, x);
  double mx = 0.0, sm = 0.0, rs = 0.0, ra = 0.0;
  float lg = 0.0f, nz = 0.0f;                 // sum of log2|x| and count over finite nonzero x
  bool nf = false;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const double a = fabs(x[q]);
    mx = fmax(mx, a);
    sm += a;
    const bool fin = a <= 1.7976931348623157e308;   // (tested alone: fmax drops a NaN)
    nf |= !fin;
    const double r = low_bits(x[q]);
    rs += r;
    ra += fabs(r);
    if (fin && a != 0.0) {
      lg += log2_abs(x[q]);
      nz += 1.0f;
    }
  }
  if (__any(nf && valid) && lane == 0) atomicOr(&p.stats[kStatNonFinite], 1u);
  __syncthreads();                            // every tile has been read
  auto at = [&](int w, int f) -> double& { return red[(w * kPartFields + f) * 64 + lane]; };
  at(wave, 0) = mx;
  at(wave, 1) = sm;
  at(wave, 2) = rs;
  at(wave, 3) = ra;
  at(wave, 4) = (double)lg;
  at(wave, 5) = (double)nz;
  __syncthreads();
  if (wave != 0 || !valid) return;
#pragma unroll
  for (int w = 1; w < kSplitWaves; ++w) {
    mx = fmax(mx, at(w, 0));
    sm += at(w, 1);
    rs += at(w, 2);
    ra += at(w, 3);
  }
  double lgd = at(0, 4), nzd = at(0, 5);
#pragma unroll
  for (int w = 1; w < kSplitWaves; ++w) {
    lgd += at(w, 4);
    nzd += at(w, 5);
  }
  const int64_t L = (int64_t)p.m + p.n;
  const int64_t fs = (int64_t)p.nslab * L;            // doubles per field
  double* q = p.part + (int64_t)blockIdx.y * L + (rows ? line : p.m + line);
  q[0] = mx;
  q[fs] = sm;
  q[2 * fs] = rs;
  q[3 * fs] = ra;
  q[4 * fs] = lgd;
  q[5 * fs] = nzd;
}

// Largest of v over the wave (v >= 0).
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

constexpr int kCombineThreads = 256;

// stats[w] = max(stats[w], v) for v >= 0 (float bits), skipped when the word
// already holds v or more: the panel's maxima settle after a few updates, so
// most blocks then issue no atomic at all (the words are read through to L2)
__device__ __forceinline__ void stat_max(uint32_t* word, float v) {
  if (!(v > 0.0f)) return;
  const uint32_t bits = __float_as_uint(v);
  if (__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= bits) return;
  atomicMax(word, bits);
}

__global__ __launch_bounds__(kCombineThreads) void split_combine_kernel(SplitArgs p) {
  const int64_t L = (int64_t)p.m + p.n;
  const int64_t line = (int64_t)blockIdx.x * kCombineThreads + threadIdx.x;
  const bool valid = line < L;
  const bool col = line >= p.m;
  float kap = 0.0f, coh = 0.0f, lam = 0.0f;
  if (valid) {
    const int64_t fs = (int64_t)p.nslab * L;
    const double* q = p.part + line;
    double mx = 0.0, sm = 0.0, rs = 0.0, ra = 0.0, lg = 0.0, nz = 0.0;
    // (unrolled: the loads of several slabs in flight; the sums stay in slab order)
#pragma unroll 4
    for (int sl = 0; sl < p.nslab; ++sl, q += L) {
      mx = fmax(mx, q[0]);
      sm += q[fs];
      rs += q[2 * fs];
      ra += q[3 * fs];
      lg += q[4 * fs];
      nz += q[5 * fs];
    }
    (col ? p.fB : p.eA)[col ? line - p.m : line] = exponent_bound(mx);
    if (nz > 0.0 && mx <= 1.7976931348623157e308)
      lam = fmaxf(log2_abs(mx) - (float)(lg / nz), 0.0f);
    if (sm > 0.0) kap = fmaxf((float)log2(mx * (double)p.w / sm), 0.0f);
    coh = coherence(rs, ra);
  }
  // the block's maxima, one per statistic and operand (a block may hold A
  // rows and B columns), then one thread folds them into the panel's
  __shared__ float bmax[kCombineThreads / 64][6];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float v[6] = {valid && !col ? kap : 0.0f, valid && col ? kap : 0.0f,
                      valid && !col ? coh : 0.0f, valid && col ? coh : 0.0f,
                      valid && !col ? lam : 0.0f, valid && col ? lam : 0.0f};
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const float w = wave_max(v[i]);
    if (lane == 0) bmax[wave][i] = w;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    constexpr int kWord[6] = {kStatKappaA, kStatKappaB, kStatCohA, kStatCohB, kStatLamA,
                              kStatLamB};
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      float m = bmax[0][i];
      for (int w = 1; w < kCombineThreads / 64; ++w) m = fmaxf(m, bmax[w][i]);
      stat_max(&p.stats[kWord[i]], m);
    }
  }
}

// The digits of one 16-k tile of one line (x scaled by 2^-e), stored at
// element `pos` of each of the first S planes.
template <int FMT, int S>
__device__ __forceinline__ void put_digits(uint8_t* dig, int64_t plane, int64_t pos,
                                           const double (&x)[16], int e) {
  constexpr int H = digit_h(FMT), T = digit_t(FMT), ESZ = digit_bytes(FMT);
  double r[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) r[q] = ldexp(x[q], -e);
  if constexpr (FMT == 2) {
    uint32_t w[kSplitMaxSlices][4];
    int8_digits<S>(r, w);
#pragma unroll
    for (int l = 0; l < S; ++l)
      *(uint4*)(dig + l * plane + pos) = make_uint4(w[l][0], w[l][1], w[l][2], w[l][3]);
    return;
  }
  int shift = H;
#pragma unroll
  for (int l = 0; l < S; ++l) {
    uint32_t w32[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const double y = ldexp(r[q], shift);
      const double d = rint(y);
      r[q] = y - d;
      if (FMT == 0)
        w32[q >> 1] |= (__float_as_uint((float)ldexp(d, -T * l)) >> 16) << (16 * (q & 1));
      else
        w32[q >> 2] |= (uint32_t)e4m3_of_int((int)d) << (8 * (q & 3));
    }
    shift = T;
    uint8_t* dst = dig + (l * plane + pos) * ESZ;
    ((uint4*)dst)[0] = make_uint4(w32[0], w32[1], w32[2], w32[3]);
    if (FMT == 0) ((uint4*)dst)[1] = make_uint4(w32[4], w32[5], w32[6], w32[7]);
  }
}

template <int FMT>
__global__ __launch_bounds__(64 * kSplitWaves) void split_digits_kernel(SplitArgs p) {
  __shared__ double tiles[kSplitWaves][64 * kTileStride];
  const int s = panel_slices(p.stats, p.fixed_s, p.smin, p.smax, p.tau_bits, p.log2k, p.log2w,
                             digit_h(FMT), digit_t(FMT));
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *p.slices_out = s;
  if (s == 0) return;                         // the FP64 kernel computes this panel
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ga = (p.m + 63) / 64;
  const bool rows = (int)blockIdx.x < ga;
  const int blk = rows ? blockIdx.x : blockIdx.x - ga;
  const int nl = rows ? p.m : p.n;
  double x[16];
  int line;
  int64_t pos;
  if constexpr (FMT == 2) {
    // INT8 planes are k32-block-major: a wave takes 32 lines x one k32 block
    // (lanes 0-31 its first 16 k, lanes 32-63 its second), so that each of
    // its plane stores is one contiguous 1 KB run
    const int l32 = lane & 31, half = lane >> 5;
    const int first = blk * 64 + (wave & 1) * 32;   // the wave's first line
    const int kb = blockIdx.y * 2 + (wave >> 1);     // k32 block (kb * 32 < Wp: Wp is a multiple of 64)
    line = first + l32;
    if (rows) {
      // the 32 x 32 tile of rows [first, first + 32) (clamped) staged through
      // this wave's LDS tile (row stride 34 doubles), 4 rows x 256 bytes per
      // wave-load, then half `half` of row l32 into x
      double* tile = tiles[wave];
      const int lr = lane >> 4, kp = 2 * (lane & 15);
      double v[16];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int row = min(first + lr + 4 * i, p.m - 1);
        const int kk = kb * 32 + kp;
        const double* rp = p.A + (int64_t)row * p.lda + p.k0 + kk;
        v[2 * i] = kk < p.w ? rp[0] : 0.0;
        v[2 * i + 1] = kk + 1 < p.w ? rp[1] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        double* t = tile + (lr + 4 * i) * 34 + kp;
        t[0] = v[2 * i];
        t[1] = v[2 * i + 1];
      }
      // the same wave reads the tile back: its LDS accesses complete in order
#pragma unroll
      for (int q = 0; q < 16; ++q) x[q] = tile[l32 * 34 + half * 16 + q];
    } else if (line < nl) {
      load_col_tile(p, line, kb * 32 + half * 16, x);
    }
    pos = (int64_t)kb * ((int64_t)nl * 32) + (int64_t)line * 32 + half * 16;
  } else {
    const int k0 = blockIdx.y * kSlabK + 16 * wave;
    if (k0 >= p.Wp) return;                   // (FP8: a half slab at the end; no barrier follows)
    line = blk * 64 + lane;
    if (rows) load_row_tile(p, blk, k0, tiles[wave], x);
    else if (line < nl) load_col_tile(p, line, k0, x);
    // k16-block-major: (plane, line, kk) at (kk / 16) lines 16 + line 16 + kk % 16
    pos = (int64_t)(k0 >> 4) * ((int64_t)nl * 16) + (int64_t)line * 16;
  }
  if (line >= nl) return;
  const int e = (rows ? p.eA : p.fB)[line];
  uint8_t* dig = (uint8_t*)(rows ? p.digA : p.digB);
  const int64_t plane = rows ? p.planeA : p.planeB;
  static_for<1, kSplitMaxSlices + 1>([&](auto S) {
    if (s == S.value) put_digits<FMT, S.value>(dig, plane, pos, x, e);
  });
}

// clears the per-panel statistics before the split of a panel
__global__ void zero_u32_kernel(uint32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// ---- BF16 slice products, streamed ------------------------------------------
// Workgroup tile 64 x 128, 4 waves (2 x 2, one per SIMD) of a 32 x 64 block
// each (two 32x32 blocks sharing the A fragment), on
// v_mfma_f32_32x32x16_bf16.  Per 16-k step the digits of every plane of the
// tile stream from global memory straight into an NS-stage LDS ring
// (buffer_load_dwordx4 ... lds through one buffer descriptor per operand,
// 6 S wave-instructions per step over the 4 waves).
// LDS image of one plane: [row][half] 16-byte units, the half index
// XOR-swizzled by bit 3 of the row so that a fragment read (32 rows x one
// half) is bank-conflict free.
//
// 32x32x16 operand layout: lane l holds A[l % 32][8 (l / 32) .. + 7] and
// B[8 (l / 32) .. + 7][l % 32]; D item v of lane l is
// D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32].
//
// Pairs (l1, l2), l1 + l2 < S, run in S rows; row r pairs A fragment
// S-1-r with B fragments 0 .. r, so every row needs one new fragment of each
// operand.  Fragment reads run LAG rows ahead of the MFMAs (one wave per
// SIMD has no other wave to hide LDS latency behind).  The step's one
// barrier sits LAG rows before its end: every read of the current stage
// has retired, so the stage is refilled by DMA for the step NS ahead (each
// load has NS - 1 steps to land), and the next stage is complete, so its
// first rows are read into the second register set while the step ends.
//
// Level accumulators (FP32): index a = l1 + l2 (0-based) for a <= 3, one
// shared accumulator for a >= 4.  Exact while a level's partial sums stay
// within 2^24: a level of a + 1 pairs of |d d'| <= 2^16 may run 256/(a+1) k.
// Each accumulator is added into the FP64 panel sum at its own cadence
// (levels 0, 1 and the shared one every 8 steps, levels 2 and 3 every 4;
// the panel is padded to a multiple of 64) and restarts from a zero C
// operand, so levels 0-3 stay exact; the shared deep accumulator (weight
// <= 2^-36) needs no exactness.
//
// The slice count S is a template parameter of the item loop (the kernel
// dispatches on the panel's count once), so the pair structure is static.
constexpr int kBf16TM = 64, kBf16TN = 128, kBf16NW = 4;
constexpr int kBf16Lds = 152 * 1024;  // LDS ring budget (bytes)
// ring depth for S planes: as many 16-k stages as fit, at most 5
constexpr int bf16_stages(int S) {
  return (kBf16Lds / (S * (kBf16TM + kBf16TN) * 32)) < 5 ? (kBf16Lds / (S * (kBf16TM + kBf16TN) * 32))
                                                          : 5;
}

// One C write of a split epilogue as exactly one vector-memory instruction,
// whatever the compiler would make of a plain store or atomic: the waits
// that follow the epilogue count these instructions.  `store`: the first
// panel of a product stores, later ones add (FP64 atomic add, no return).
__device__ __forceinline__ void c_write(double* dst, double v, int store) {
  if (store) asm volatile("global_store_dwordx2 %0, %1, off" ::"v"(dst), "v"(v) : "memory");
  else asm volatile("global_atomic_add_f64 %0, %1, off" ::"v"(dst), "v"(v) : "memory");
}

// Wait until at most k x PER of this wave's vector-memory instructions are
// outstanding (k <= KMAX, known only at run time; the count is an immediate).
template <int PER, int KMAX>
__device__ __forceinline__ void vm_wait_steps(int k) {
  if (KMAX >= 4 && k >= 4) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(4 * PER) : "memory");
  else if (KMAX >= 3 && k == 3) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(3 * PER) : "memory");
  else if (KMAX >= 2 && k == 2) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(2 * PER) : "memory");
  else if (KMAX >= 1 && k == 1) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(PER) : "memory");
  else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// Wait until at most k x PER + EXTRA of this wave's vector-memory
// instructions are outstanding (k <= KMAX at run time; the count is an
// immediate, capped at the counter's 63).
template <int PER, int KMAX, int EXTRA>
__device__ __forceinline__ void vm_wait_steps_plus(int k) {
  if (KMAX >= 4 && k >= 4) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(min(63, 4 * PER + EXTRA)) : "memory");
  else if (KMAX >= 3 && k == 3) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(min(63, 3 * PER + EXTRA)) : "memory");
  else if (KMAX >= 2 && k == 2) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(min(63, 2 * PER + EXTRA)) : "memory");
  else if (KMAX >= 1 && k == 1) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(min(63, PER + EXTRA)) : "memory");
  else asm volatile("s_waitcnt vmcnt(%0)" ::"n"(min(63, EXTRA)) : "memory");
}

template <int S>
__device__ __forceinline__ void slice_bf16_items(const SliceArgs& p, uint8_t* smem) {
  constexpr int TM = kBf16TM, TN = kBf16TN, NW = kBf16NW, NS = bf16_stages(S);
  constexpr int ABYTES = S * TM * 32, BBYTES = S * TN * 32, SB = ABYTES + BBYTES;
  // DMA wave-instructions per 16-k step of waves 0-1 and 2-3
  constexpr int NIHI = 3 * (S / 2) + (S & 1 ? 2 : 0), NILO = 3 * (S / 2) + (S & 1);
  constexpr int NACC = S < 5 ? S : 5;
  // rows of fragment reads ahead of the MFMAs (2 measured best up to 5 planes, 3 above)
  constexpr int LAG = S < 3 ? S : (S <= 5 ? 2 : 3);
  static_assert(NS >= 3 && NS * SB <= kBf16Lds, "LDS ring");

  constexpr int NSTORE = 32;                    // C writes per lane and item (2 x 16)
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform
  const int wm = wave >> 1, wn = wave & 1;
  const bool hi = wave < 2;                     // this wave issues NIHI per step
  // Per-lane offsets come from a lane id read where they are needed, opaque
  // to the compiler (v_mbcnt): derived once, they would stay live across
  // the epilogue and be spilled, and a scratch reload after the next item's
  // DMA would wait for that DMA and the epilogue's writes.
  auto lane_id = [] {
    int l;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
    return l;
  };

  const __amdgpu_buffer_rsrc_t rsrcA =
      __builtin_amdgcn_make_buffer_rsrc((void*)p.digA, (short)0, (int)p.bytesA, kBufferWord3);
  const __amdgpu_buffer_rsrc_t rsrcB =
      __builtin_amdgcn_make_buffer_rsrc((void*)p.digB, (short)0, (int)p.bytesB, kBufferWord3);
  const uint32_t kbA = (uint32_t)p.rowsA * 32u, kbB = (uint32_t)p.rowsB * 32u;  // bytes per k16 block
  const uint32_t planeAB = (uint32_t)(p.planeA * 2), planeBB = (uint32_t)(p.planeB * 2);
  const int nsteps = p.Wp / 16;                // a multiple of 4
  // LDS byte offsets of this lane's A and B fragments (block 1 is 32
  // columns on: same swizzle bit)
  auto frag_offsets = [&](int& aoff, int& boff) {
    const int l = lane_id(), l32 = l & 31, lh = l >> 5;
    const int arow = wm * 32 + l32, bcol = wn * 64 + l32;
    aoff = (arow * 2 + (lh ^ ((arow >> 3) & 1))) * 16;
    boff = (bcol * 2 + (lh ^ ((bcol >> 3) & 1))) * 16;
  };

  const int bid = blockIdx.x, xcd = bid & 7, slot0 = bid >> 3;
  const int slots = p.persistent ? (gridDim.x + 7 - xcd) >> 3 : 1;
  // the work item of a slot of this workgroup, or -1
  auto item_index = [&](int slot) {
    if (!p.persistent && slot != slot0) return -1;
    if (slot >= p.per_xcd) return -1;
    const int idx = xcd * p.per_xcd + slot;
    return idx < p.nitems ? idx : -1;
  };

    // DMA: a 16-k step moves, per plane, 2 wave-instructions of A (64 rows x
    // 32 bytes) and 4 of B (128 columns x 32 bytes), 64 16-byte units each
    // (unit u = row or column u/2, half u%2).  Per pair of planes (l, l+1)
    // wave w loads A half w%2 of plane l + w/2 and B quarter w of both
    // planes; an odd last plane gives its A halves to waves 0, 1.  So each
    // wave has one per-lane byte offset into A and one into B (ragged rows
    // and columns clamped to the last valid one); plane and k16 block are a
    // uniform offset in the buffer descriptor's soffset.
  uint32_t voffA = 0, voffB = 0;
  auto set_dma_offsets = [&](const WorkItem& w) {
    const int l = lane_id();
    const int ua = (wave & 1) * 64 + l;
    const int rowa = ua >> 1, halfa = (ua & 1) ^ ((rowa >> 3) & 1);
    const int ub = wave * 64 + l;
    const int colb = ub >> 1, halfb = (ub & 1) ^ ((colb >> 3) & 1);
    voffA = (uint32_t)(w.r0 + min(rowa, w.h - 1)) * 32u + halfa * 16u;
    voffB = (uint32_t)(w.c0 + min(colb, w.w - 1)) * 32u + halfb * 16u;
  };
    auto dmaA = [&](int plane, int kb, uint8_t* dst) {
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rsrcA, (__attribute__((address_space(3))) void*)dst, 16, voffA,
          (uint32_t)(plane * planeAB + kb * kbA), 0, 0);
    };
    auto dmaB = [&](int plane, int kb, uint8_t* dst) {
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rsrcB, (__attribute__((address_space(3))) void*)dst, 16, voffB,
          (uint32_t)(plane * planeBB + kb * kbB), 0, 0);
    };
    auto issue = [&](int kb, int st) {
      uint8_t* stage = smem + st * SB;
#pragma unroll
      for (int l = 0; l + 1 < S; l += 2) {
        const int pa = l + (wave >> 1);
        dmaA(pa, kb, stage + pa * (TM * 32) + (wave & 1) * 1024);
        dmaB(l, kb, stage + ABYTES + l * (TN * 32) + wave * 1024);
        dmaB(l + 1, kb, stage + ABYTES + (l + 1) * (TN * 32) + wave * 1024);
      }
      if (S & 1) {
        if (wave < 2) dmaA(S - 1, kb, stage + (S - 1) * (TM * 32) + wave * 1024);
        dmaB(S - 1, kb, stage + ABYTES + (S - 1) * (TN * 32) + wave * 1024);
      }
    };
    // wait for this wave's loads of step s, with `later` steps issued after it
    auto wait_step = [&](int later) {
      if (hi) vm_wait_steps<NIHI, NS - 1>(later);
      else vm_wait_steps<NILO, NS - 1>(later);
    };

  int idx = item_index(slot0);
  if (idx < 0) return;
  WorkItem it = p.items[idx];
  set_dma_offsets(it);

  // Fragments.  Rows run in the order r = 0 .. S-1, row r pairing A
  // fragment S-1-r with B fragments 0 .. r, so each row needs one new A and
  // one new B fragment (per block).  Reads run LAG rows ahead of the MFMAs;
  // the last LAG rows of a step read the first LAG rows of the next step
  // (or item) into the other register set.
  bf8v fa[2][S], fb0[2][S], fb1[2][S];
  int aoff, boff;
  auto read_row = [&](int set, int st, int r) {
    const uint8_t* sA = smem + st * SB;
    const uint8_t* sB = sA + ABYTES;
    fa[set][S - 1 - r] = *(const bf8v*)(sA + (S - 1 - r) * (TM * 32) + aoff);
    fb0[set][r] = *(const bf8v*)(sB + r * (TN * 32) + boff);
    fb1[set][r] = *(const bf8v*)(sB + r * (TN * 32) + boff + 1024);
  };
  // the first item's prologue: NS steps in flight, step 0 landed, the first
  // LAG rows of fragments read
#pragma unroll
  for (int st = 0; st < NS; ++st)
    if (st < nsteps) issue(st, st);
  wait_step(min(NS - 1, nsteps - 1));
  ring_barrier();
  frag_offsets(aoff, boff);
#pragma unroll
  for (int r = 0; r < LAG; ++r) read_row(0, 0, r);

  for (int slot = slot0; idx >= 0; slot += slots) {
    f16v acc0[NACC], acc1[NACC];               // level accumulators, blocks 0 and 1
    double cp0[16], cp1[16];                   // FP64 panel sums
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      cp0[v] = 0.0;
      cp1[v] = 0.0;
    }
    // In the first step of a group of four every accumulator starts from
    // zero: its first pair (row S-1-a, or row 0 for the shared deep one, with
    // l2 = 0) takes a zero C operand.
    const f16v zero = {};
    auto row = [&](int set, int r, int restart) {
      const int l1 = S - 1 - r;
#pragma unroll
      for (int l2 = 0; l2 <= r; ++l2) {
        const int a = (l1 + l2) < NACC - 1 ? (l1 + l2) : NACC - 1;
        const bool z = ((restart >> a) & 1) && l2 == 0 && r == (a == NACC - 1 ? 0 : S - 1 - a);
        acc0[a] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[set][l1], fb0[set][l2], z ? zero : acc0[a],
                                                          0, 0, 0);
        acc1[a] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[set][l1], fb1[set][l2], z ? zero : acc1[a],
                                                          0, 0, 0);
      }
    };
    // Accumulator a is added into the FP64 panel sum every per(a) steps and
    // then restarts from a zero C operand: every 8 steps (128 k) for levels
    // 0 and 1 and the shared deep one, every 4 for levels 2 and 3, each
    // within its exactness bound (level a may run 256/(a+1) k).  A flush adds
    // the levels in the order of decreasing weight.  Runs of 8 steps are
    // unrolled so that every flush and restart is static (longer runs raise
    // the register pressure past the file); a remaining 4 steps flush every
    // level.
    auto flush = [&](int mask) {
#pragma unroll
      for (int a = 0; a < NACC; ++a)
        if ((mask >> a) & 1) {
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            cp0[v] += (double)acc0[a][v];
            cp1[v] += (double)acc1[a][v];
          }
        }
    };
    // one 16-k step: fragments of step ci are in set `cur`.  The barrier sits
    // before row S-LAG: by then every fragment of step ci has been read
    // (ring_barrier retires the reads), so stage ci is free for the DMA of
    // step ci+NS, and stage ci+1 is complete for every wave.
    auto step = [&](int ci, int cur, int restart) {
      const int nxt = cur ^ 1;
      const bool more = ci + 1 < nsteps;
#pragma unroll
      for (int r = 0; r < S; ++r) {
        if (r == S - LAG && more) {
          wait_step(min(NS - 2, nsteps - 2 - ci));   // step ci + 1 landed (this wave)
          ring_barrier();
          if (ci + NS < nsteps) issue(ci + NS, ci % NS);
        }
        if (r + LAG < S) read_row(cur, ci % NS, r + LAG);
        else if (more) read_row(nxt, (ci + 1) % NS, r + LAG - S);
        row(cur, r, restart);
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    constexpr int ALL = (1 << NACC) - 1;
    // levels whose run starts (ends) at step j of an 8-step run
    auto per = [](int a) { return a <= 1 || a >= 4 ? 8 : 4; };
    auto starts = [&](int j) {
      int m = 0;
      for (int a = 0; a < NACC; ++a) m |= (j % per(a) == 0) << a;
      return m;
    };
    auto ends = [&](int j) {
      int m = 0;
      for (int a = 0; a < NACC; ++a) m |= ((j + 1) % per(a) == 0) << a;
      return m;
    };

    int ci = 0;
    for (; ci + 8 <= nsteps; ci += 8) {
      static_for<0, 8>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        step(ci + j, j & 1, starts(j));
        flush(ends(j));
        __builtin_amdgcn_sched_barrier(0);
      });
    }
    for (; ci < nsteps; ci += 4) {
      step(ci, 0, ALL);
      step(ci + 1, 1, 0);
      step(ci + 2, 0, 0);
      step(ci + 3, 1, 0);
      flush(ALL);
    }

    // Epilogue (as in the INT8 kernel): (1) the exponent loads; (2) once they
    // have landed and every wave is done with the ring, the next item's first
    // NS steps of DMA; (3) C += 2^(e_i + f_j - 16) x panel sum as FP64
    // atomic adds (the first panel of a product stores instead): no wave
    // waits for C, each C element gets exactly one add per launch, so the
    // result is the single rounded sum a load and a store would give, and
    // the next item's first wait leaves these NSTORE writes in flight.
    const int lane_e = lane_id();
    const int le32 = lane_e & 31, leh = lane_e >> 5;
    auto erow = [&](int v) { return wm * 32 + 8 * (v >> 2) + 4 * leh + (v & 3); };
    int ea[16], fq[2];
#pragma unroll
    for (int v = 0; v < 16; ++v) ea[v] = p.eA[it.r0 + min(erow(v), it.h - 1)];
#pragma unroll
    for (int q = 0; q < 2; ++q) fq[q] = p.fB[it.c0 + min(wn * 64 + q * 32 + le32, it.w - 1)];
    // the exponents have landed before the DMA is issued (vmcnt(0), an
    // S_WAITCNT the compiler sees), so that no wait for them after it can
    // hold the DMA too
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __builtin_amdgcn_sched_barrier(0);
    // every wave's reads of the ring have retired, and no DMA of this item is
    // outstanding
    ring_barrier();
    const int nidx = __builtin_amdgcn_readfirstlane(item_index(slot + slots));
    WorkItem nt = it;
    if (nidx >= 0) {
      nt = p.items[nidx];
      set_dma_offsets(nt);
#pragma unroll
      for (int st = 0; st < NS; ++st)
        if (st < nsteps) issue(st, st);
    }
    __builtin_amdgcn_sched_barrier(0);
    // Every lane issues all NSTORE writes, each one instruction (c_write):
    // lanes outside a ragged item write to their own slot of the dump area,
    // so that the count the next item's first wait allows for is exact.
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int col = wn * 64 + q * 32 + le32;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = erow(v);
        const double add = ldexp(q ? cp1[v] : cp0[v], ea[v] + fq[q] - 16);
        const bool in = row < it.h && col < it.w;
        double* dst = in ? p.C + (int64_t)(it.r0 + row) * p.ldc + it.c0 + col : p.dump + lane_e;
        c_write(dst, add, p.zero_init);
      }
    }
    it = nt;
    idx = nidx;
    if (idx >= 0) {
      // the next item's step 0 landed; its writes above are the newest
      // NSTORE vector-memory instructions and need not have completed
      if (hi) vm_wait_steps_plus<NIHI, NS - 1, NSTORE>(min(NS - 1, nsteps - 1));
      else vm_wait_steps_plus<NILO, NS - 1, NSTORE>(min(NS - 1, nsteps - 1));
      ring_barrier();
      frag_offsets(aoff, boff);
#pragma unroll
      for (int r = 0; r < LAG; ++r) read_row(0, 0, r);
    }
  }
}

__global__ __launch_bounds__(256, 1) void slice_bf16_kernel(SliceArgs p) {
  __shared__ __attribute__((aligned(1024))) uint8_t smem[kBf16Lds];
  const int s = *p.slices;
  if (s <= 0) return;                          // the FP64 kernel computes this panel
  switch (s) {
    case 1: slice_bf16_items<1>(p, smem); break;
    case 2: slice_bf16_items<2>(p, smem); break;
    case 3: slice_bf16_items<3>(p, smem); break;
    case 4: slice_bf16_items<4>(p, smem); break;
    case 5: slice_bf16_items<5>(p, smem); break;
    case 6: slice_bf16_items<6>(p, smem); break;
    default: slice_bf16_items<7>(p, smem); break;
  }
}

// ---- FP8 slice products, streamed -------------------------------------------
// The BF16 kernel's design with e4m3 digits on v_mfma_f32_32x32x16_fp8_fp8
// (lane l holds A[l % 32][8 (l / 32) .. + 7] and B[8 (l / 32) .. + 7][l % 32],
// 8 bytes each; D as for the BF16 instruction).  Per 16-k step a plane is 64
// rows x 16 bytes of A (one wave-instruction of 64 16-byte units) and
// 128 x 16 bytes of B (two), so a step is 3 S wave-instructions, dealt
// round-robin over the 4 waves.  A plane's LDS image is its HBM layout
// ([row][16 bytes]); a fragment read (32 rows x 16 bytes) is 512 contiguous
// bytes, free of bank conflicts.  Every level of e4m3 digit pairs stays
// exact in FP32 over a whole panel (at most 7 pairs of |d d'| <= 2^8 per k,
// panels of at most 8192 k), so each level keeps its own accumulator from
// the item's first step to its last and is added into FP64 once, scaled by
// 2^(-5 a), smallest weight first.
constexpr int kFp8Lds = 152 * 1024;   // LDS ring budget (bytes)
constexpr int fp8_stages(int S) {
  return kFp8Lds / (S * 192 * 16) < 5 ? kFp8Lds / (S * 192 * 16) : 5;
}

template <int S>
__device__ __forceinline__ void slice_fp8_items(const SliceArgs& p, uint8_t* smem) {
  constexpr int TM = 64, TN = 128, NS = fp8_stages(S);
  constexpr int ABYTES = S * TM * 16, BBYTES = S * TN * 16, SB = ABYTES + BBYTES;
  constexpr int NI = 3 * S;                           // wave-instructions per step
  constexpr int NILO = NI / 4, NIHI = NILO + (NI % 4 ? 1 : 0);
  constexpr int LAG = S < 3 ? S : (S <= 5 ? 2 : 3);   // rows of reads ahead of the MFMAs
  constexpr int H = 4, T = 5;
  static_assert(NS >= 3 && NS * SB <= kFp8Lds, "LDS ring");

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform
  const int wm = wave >> 1, wn = wave & 1;
  const int l32 = lane & 31, lh = lane >> 5;
  const bool hi = wave < NI % 4;                // this wave issues NIHI per step

  const __amdgpu_buffer_rsrc_t rsrcA =
      __builtin_amdgcn_make_buffer_rsrc((void*)p.digA, (short)0, (int)p.bytesA, kBufferWord3);
  const __amdgpu_buffer_rsrc_t rsrcB =
      __builtin_amdgcn_make_buffer_rsrc((void*)p.digB, (short)0, (int)p.bytesB, kBufferWord3);
  const uint32_t kbA = (uint32_t)p.rowsA * 16u, kbB = (uint32_t)p.rowsB * 16u;  // per k16 block
  const uint32_t planeAB = (uint32_t)p.planeA, planeBB = (uint32_t)p.planeB;   // 1-byte digits
  const int nsteps = p.Wp / 16;                // even: the panel is padded to 32 k
  const int aoff = (wm * 32 + l32) * 16 + lh * 8;
  const int boff = (wn * 64 + l32) * 16 + lh * 8;   // block 1: 32 columns (512 bytes) on

  const int bid = blockIdx.x, xcd = bid & 7, slot0 = bid >> 3;
  const int slots = p.persistent ? (gridDim.x + 7 - xcd) >> 3 : 1;

  for (int slot = slot0;; slot += slots) {
    if (!p.persistent && slot != slot0) break;
    if (slot >= p.per_xcd) break;
    const int idx = xcd * p.per_xcd + slot;
    if (idx >= p.nitems) break;
    const WorkItem it = p.items[idx];

    // per-lane byte offsets of the lane's row of A and columns of B (ragged
    // edges clamped to the last valid one); plane and k16 block are uniform
    const uint32_t voffA = (uint32_t)(it.r0 + min(lane, it.h - 1)) * 16u;
    const uint32_t voffB0 = (uint32_t)(it.c0 + min(lane, it.w - 1)) * 16u;
    const uint32_t voffB1 = (uint32_t)(it.c0 + min(64 + lane, it.w - 1)) * 16u;
    auto dma = [&](__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, uint8_t* dst) {
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          r, (__attribute__((address_space(3))) void*)dst, 16, voff, soff, 0, 0);
    };
    // instruction i of a step: plane i / 3; A (i % 3 == 0) or B columns
    // 0..63 / 64..127; issued by wave i % 4, so a wave walks i = wave,
    // wave + 4, ... (a uniform loop: unrolled over every instruction and
    // stage, the scalar offsets alone spill the scalar file)
    auto issue = [&](int kb, int st) {
      uint8_t* stage = smem + st * SB;
      const int cnt = hi ? NIHI : NILO;
#pragma unroll 1
      for (int j = 0; j < cnt; ++j) {
        const int i = wave + 4 * j;
        const int l = i / 3, kind = i - 3 * l;
        if (kind == 0)
          dma(rsrcA, voffA, (uint32_t)(l * planeAB + kb * kbA), stage + l * (TM * 16));
        else
          dma(rsrcB, kind == 1 ? voffB0 : voffB1, (uint32_t)(l * planeBB + kb * kbB),
              stage + ABYTES + l * (TN * 16) + (kind - 1) * 1024);
      }
    };
    auto wait_step = [&](int later) {
      if (hi) vm_wait_steps<NIHI, NS - 1>(later);
      else vm_wait_steps<NILO, NS - 1>(later);
    };

    f16v acc0[S], acc1[S];                     // one accumulator per level, blocks 0 and 1
    // fragments: row r pairs A plane S-1-r with B planes 0 .. r; reads run LAG
    // rows ahead, the last LAG rows of a step reading the next step's first
    // rows into the other register set
    long fa[2][S], fb0[2][S], fb1[2][S];
    auto read_row = [&](int set, int st, int r) {
      const uint8_t* sA = smem + st * SB;
      const uint8_t* sB = sA + ABYTES;
      fa[set][S - 1 - r] = *(const long*)(sA + (S - 1 - r) * (TM * 16) + aoff);
      fb0[set][r] = *(const long*)(sB + r * (TN * 16) + boff);
      fb1[set][r] = *(const long*)(sB + r * (TN * 16) + boff + 512);
    };
    // in the item's first step each level's first pair (row S-1-a, l2 = 0)
    // takes a zero C operand
    const f16v zero = {};
    auto row = [&](int set, int r, bool first) {
      const int l1 = S - 1 - r;
#pragma unroll
      for (int l2 = 0; l2 <= r; ++l2) {
        const int a = l1 + l2;
        const bool z = first && l2 == 0;
        acc0[a] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(fa[set][l1], fb0[set][l2],
                                                             z ? zero : acc0[a], 0, 0, 0);
        acc1[a] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(fa[set][l1], fb1[set][l2],
                                                             z ? zero : acc1[a], 0, 0, 0);
      }
    };
    auto step = [&](int ci, int cur, bool first) {
      const int nxt = cur ^ 1;
      const bool more = ci + 1 < nsteps;
#pragma unroll
      for (int r = 0; r < S; ++r) {
        if (r == S - LAG && more) {
          wait_step(min(NS - 2, nsteps - 2 - ci));   // step ci + 1 landed (this wave)
          ring_barrier();
          if (ci + NS < nsteps) issue(ci + NS, ci % NS);
        }
        if (r + LAG < S) read_row(cur, ci % NS, r + LAG);
        else if (more) read_row(nxt, (ci + 1) % NS, r + LAG - S);
        row(cur, r, first);
        __builtin_amdgcn_sched_barrier(0);
      }
    };

#pragma unroll
    for (int st = 0; st < NS; ++st)
      if (st < nsteps) issue(st, st);
    wait_step(min(NS - 1, nsteps - 1));
    ring_barrier();
#pragma unroll
    for (int r = 0; r < LAG; ++r) read_row(0, 0, r);
    step(0, 0, true);
    int ci = 1;
    for (; ci + 2 <= nsteps; ci += 2) {
      step(ci, 1, false);
      step(ci + 1, 0, false);
    }
    if (ci < nsteps) step(ci, 1, false);
    __syncthreads();  // the ring is reused by the next item

    double cp0[16], cp1[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      cp0[v] = 0.0;
      cp1[v] = 0.0;
    }
#pragma unroll
    for (int a = S - 1; a >= 0; --a) {
      const double wgt = ldexp(1.0, -T * a);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        cp0[v] = fma((double)acc0[a][v], wgt, cp0[v]);
        cp1[v] = fma((double)acc1[a][v], wgt, cp1[v]);
      }
    }

    // C += 2^(e_i + f_j - 2H) x panel sum (clamped loads, predicated stores).
    // The lane's rows and columns are derived afresh from an opaque lane id:
    // hoisted out of the item loop they stay live across it and spill.
    int lane_e;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(lane_e));
    const int l32e = lane_e & 31, lhe = lane_e >> 5;
    auto erow_e = [&](int v) { return wm * 32 + 8 * (v >> 2) + 4 * lhe + (v & 3); };
    int ea[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) ea[v] = p.eA[it.r0 + min(erow_e(v), it.h - 1)];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int col = wn * 64 + q * 32 + l32e;
      const int fq = p.fB[it.c0 + min(col, it.w - 1)];
      double cold[16];
      if (!p.zero_init) {
#pragma unroll
        for (int v = 0; v < 16; ++v)
          cold[v] = p.C[(int64_t)(it.r0 + min(erow_e(v), it.h - 1)) * p.ldc + it.c0 +
                        min(col, it.w - 1)];
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = erow_e(v);
        const double add = ldexp(q ? cp1[v] : cp0[v], ea[v] + fq - 2 * H);
        if (row < it.h && col < it.w)
          p.C[(int64_t)(it.r0 + row) * p.ldc + it.c0 + col] = p.zero_init ? add : cold[v] + add;
      }
    }
  }
}

__global__ __launch_bounds__(256, 1) void slice_fp8_kernel(SliceArgs p) {
  __shared__ __attribute__((aligned(1024))) uint8_t smem[kFp8Lds];
  const int s = *p.slices;
  if (s <= 0) return;                          // the FP64 kernel computes this panel
  switch (s) {
    case 1: slice_fp8_items<1>(p, smem); break;
    case 2: slice_fp8_items<2>(p, smem); break;
    case 3: slice_fp8_items<3>(p, smem); break;
    case 4: slice_fp8_items<4>(p, smem); break;
    case 5: slice_fp8_items<5>(p, smem); break;
    case 6: slice_fp8_items<6>(p, smem); break;
    default: slice_fp8_items<7>(p, smem); break;
  }
}

// ---- INT8 slice products, streamed ------------------------------------------
// The BF16 kernel's data flow on INT8 digits and v_mfma_i32_32x32x32_i8: lane
// l holds A[l % 32][16 (l / 32) .. + 15] and B[16 (l / 32) .. + 15][l % 32]
// (16 bytes each), D item v of lane l is D[8 (v / 4) + 4 (l / 32) + v % 4]
// [l % 32] in INT32.  On gfx950 the instruction issues in the time of the
// 16-k BF16 one from the same 16 bytes per lane, so it does twice the k per
// clock; a 32-k step of a plane is the BF16 step's 64 x 32 bytes of A and
// 128 x 32 bytes of B, with the same LDS image, swizzle, ring and DMA
// deal over the waves.  The planes are stored k32-block-major: the
// 16-byte unit (row, half) of a 32-k step sits at row x 32 + half x 16 past
// the step's base, so each DMA wave-instruction (32 rows or columns, both
// halves) reads one contiguous 1 KB run (with k16 blocks it read two 512-byte
// runs a k16 block apart).  Every level of digit pairs stays exact in INT32
// over a whole panel (at most 8 pairs of |d d'| <= 2^14 per k, panels of at
// most 8192 k), so each level keeps one accumulator from the item's first
// step to its last, with no restarts, and the levels are added into FP64
// once, scaled by 2^(-8 a), smallest weight first.  The results go into C
// as FP64 atomic adds issued after the next item's first steps of DMA (see
// the epilogue), so that no wave waits for C and the next item's first
// wait can leave the writes in flight.

template <int S>
__device__ __forceinline__ void slice_i8_items(const SliceArgs& p, uint8_t* smem) {
  constexpr int TM = kBf16TM, TN = kBf16TN, NS = bf16_stages(S);
  constexpr int ABYTES = S * TM * 32, BBYTES = S * TN * 32, SB = ABYTES + BBYTES;
  // DMA wave-instructions per 32-k step of waves 0-1 and 2-3
  constexpr int NIHI = 3 * (S / 2) + (S & 1 ? 2 : 0), NILO = 3 * (S / 2) + (S & 1);
  // rows of fragment reads ahead of the MFMAs: 2 (at s = 8, 1.5 % faster than 3;
  // even at s = 6)
  constexpr int LAG = S < 3 ? S : 2;
  constexpr int NSTORE = 32;                    // C writes per lane and item (2 x 16)
  static_assert(NS >= 3 && NS * SB <= kBf16Lds, "LDS ring");

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform
  const int wm = wave >> 1, wn = wave & 1;
  const bool hi = wave < 2;                     // this wave issues NIHI per step
  // Per-lane offsets are derived from a lane id read where they are needed,
  // opaque to the compiler (v_mbcnt): derived once, they stay live across
  // the epilogue, where 8 levels of accumulators leave no room, and their
  // reloads from scratch would wait for the epilogue's writes.
  auto lane_id = [] {
    int l;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
    return l;
  };

  const __amdgpu_buffer_rsrc_t rsrcA =
      __builtin_amdgcn_make_buffer_rsrc((void*)p.digA, (short)0, (int)p.bytesA, kBufferWord3);
  const __amdgpu_buffer_rsrc_t rsrcB =
      __builtin_amdgcn_make_buffer_rsrc((void*)p.digB, (short)0, (int)p.bytesB, kBufferWord3);
  const uint32_t kbA = (uint32_t)p.rowsA * 32u, kbB = (uint32_t)p.rowsB * 32u;  // bytes per 32-k step
  const uint32_t planeAB = (uint32_t)p.planeA, planeBB = (uint32_t)p.planeB;   // one byte per digit
  const int nsteps = p.Wp / 32;                // even: the panel is padded to 64 k
  // LDS byte offsets of this lane's A and B fragments (rows / columns
  // 32 wm + l % 32 and 64 wn + l % 32, half l / 32, swizzled)
  auto frag_offsets = [&](int& aoff, int& boff) {
    const int l = lane_id(), l32 = l & 31, lh = l >> 5;
    const int arow = wm * 32 + l32, bcol = wn * 64 + l32;
    aoff = (arow * 2 + (lh ^ ((arow >> 3) & 1))) * 16;
    boff = (bcol * 2 + (lh ^ ((bcol >> 3) & 1))) * 16;
  };

  const int bid = blockIdx.x, xcd = bid & 7, slot0 = bid >> 3;
  const int slots = p.persistent ? (gridDim.x + 7 - xcd) >> 3 : 1;
  // the work item of the k-th slot of this workgroup, or -1
  auto item_index = [&](int slot) {
    if (!p.persistent && slot != slot0) return -1;
    if (slot >= p.per_xcd) return -1;
    const int idx = xcd * p.per_xcd + slot;
    return idx < p.nitems ? idx : -1;
  };

  // the BF16 kernel's deal of LDS units over the waves; only the global
  // offset of a unit differs (ragged rows and columns clamped)
  uint32_t voffA = 0, voffB = 0;
  auto set_dma_offsets = [&](const WorkItem& w) {
    const int l = lane_id();
    const int ua = (wave & 1) * 64 + l;
    const int rowa = ua >> 1, halfa = (ua & 1) ^ ((rowa >> 3) & 1);
    const int ub = wave * 64 + l;
    const int colb = ub >> 1, halfb = (ub & 1) ^ ((colb >> 3) & 1);
    voffA = (uint32_t)(w.r0 + min(rowa, w.h - 1)) * 32u + halfa * 16u;
    voffB = (uint32_t)(w.c0 + min(colb, w.w - 1)) * 32u + halfb * 16u;
  };
  auto dmaA = [&](int plane, int kb, uint8_t* dst) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrcA, (__attribute__((address_space(3))) void*)dst, 16,
                                             voffA, (uint32_t)(plane * planeAB + kb * kbA), 0, 0);
  };
  auto dmaB = [&](int plane, int kb, uint8_t* dst) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrcB, (__attribute__((address_space(3))) void*)dst, 16,
                                             voffB, (uint32_t)(plane * planeBB + kb * kbB), 0, 0);
  };
  auto issue = [&](int kb, int st) {
    uint8_t* stage = smem + st * SB;
#pragma unroll
    for (int l = 0; l + 1 < S; l += 2) {
      const int pa = l + (wave >> 1);
      dmaA(pa, kb, stage + pa * (TM * 32) + (wave & 1) * 1024);
      dmaB(l, kb, stage + ABYTES + l * (TN * 32) + wave * 1024);
      dmaB(l + 1, kb, stage + ABYTES + (l + 1) * (TN * 32) + wave * 1024);
    }
    if (S & 1) {
      if (wave < 2) dmaA(S - 1, kb, stage + (S - 1) * (TM * 32) + wave * 1024);
      dmaB(S - 1, kb, stage + ABYTES + (S - 1) * (TN * 32) + wave * 1024);
    }
  };
  auto wait_step = [&](int later) {
    if (hi) vm_wait_steps<NIHI, NS - 1>(later);
    else vm_wait_steps<NILO, NS - 1>(later);
  };

  int idx = item_index(slot0);
  if (idx < 0) return;
  WorkItem it = p.items[idx];
  set_dma_offsets(it);
  i4v fa[2][S], fb0[2][S], fb1[2][S];          // fragments, two register sets
  int aoff, boff;
  auto read_row = [&](int set, int st, int r) {
    const uint8_t* sA = smem + st * SB;
    const uint8_t* sB = sA + ABYTES;
    fa[set][S - 1 - r] = *(const i4v*)(sA + (S - 1 - r) * (TM * 32) + aoff);
    fb0[set][r] = *(const i4v*)(sB + r * (TN * 32) + boff);
    fb1[set][r] = *(const i4v*)(sB + r * (TN * 32) + boff + 1024);
  };
  // the first item's prologue: NS steps in flight, step 0 landed, the first
  // LAG rows of fragments read
#pragma unroll
  for (int st = 0; st < NS; ++st)
    if (st < nsteps) issue(st, st);
  wait_step(min(NS - 1, nsteps - 1));
  ring_barrier();
  frag_offsets(aoff, boff);
#pragma unroll
  for (int r = 0; r < LAG; ++r) read_row(0, 0, r);

  for (int slot = slot0; idx >= 0; slot += slots) {
    i16v acc0[S], acc1[S];                     // level accumulators, blocks 0 and 1
#pragma unroll
    for (int a = 0; a < S; ++a) {
      acc0[a] = i16v{};
      acc1[a] = i16v{};
    }

    // rows r = 0 .. S-1 pair A fragment S-1-r with B fragments 0 .. r; reads
    // run LAG rows ahead of the MFMAs (as in the BF16 kernel)
    auto row = [&](int set, int r) {
      const int l1 = S - 1 - r;
#pragma unroll
      for (int l2 = 0; l2 <= r; ++l2) {
        const int a = l1 + l2;
        acc0[a] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[set][l1], fb0[set][l2], acc0[a], 0, 0, 0);
        acc1[a] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[set][l1], fb1[set][l2], acc1[a], 0, 0, 0);
      }
    };
    // one 32-k step, with the BF16 kernel's barrier placement and refill
    auto step = [&](int ci, int cur) {
      const int nxt = cur ^ 1;
      const bool more = ci + 1 < nsteps;
#pragma unroll
      for (int r = 0; r < S; ++r) {
        if (r == S - LAG && more) {
          wait_step(min(NS - 2, nsteps - 2 - ci));   // step ci + 1 landed (this wave)
          ring_barrier();
          if (ci + NS < nsteps) issue(ci + NS, ci % NS);
        }
        if (r + LAG < S) read_row(cur, ci % NS, r + LAG);
        else if (more) read_row(nxt, (ci + 1) % NS, r + LAG - S);
        row(cur, r);
        __builtin_amdgcn_sched_barrier(0);
      }
    };

    for (int ci = 0; ci < nsteps; ci += 2) {
      step(ci, 0);
      step(ci + 1, 1);
    }

    // Epilogue: (1) the exponent loads; (2) once every wave is done with the
    // ring, the next item's first NS steps of DMA; (3) per C element the
    // level sum, sum_a 2^(-8 a) level_a from the smallest weight up (Horner
    // in 2^-8: every scaling is exact; taken before the DMA), and
    // C += 2^(e_i + f_j - 12) x sum as
    // an FP64 atomic add (the first panel of a product stores instead): the
    // read of C happens in L2, no wave waits for it, and each C element gets
    // exactly one add per launch, so the result is the single rounded sum a
    // load and a store would give.  The next item's first wait leaves these
    // NSTORE writes in flight.  The lane id is read again here, opaque to
    // the compiler: derived from the kernel's lane id, the 16 row indices
    // below are hoisted out of the item loop and spilled.
    const int lane_e = lane_id();
    const int le32 = lane_e & 31, leh = lane_e >> 5;
    auto erow = [&](int v) { return wm * 32 + 8 * (v >> 2) + 4 * leh + (v & 3); };
    int ea[16], fq[2];
#pragma unroll
    for (int v = 0; v < 16; ++v) ea[v] = p.eA[it.r0 + min(erow(v), it.h - 1)];
#pragma unroll
    for (int q = 0; q < 2; ++q) fq[q] = p.fB[it.c0 + min(wn * 64 + q * 32 + le32, it.w - 1)];
    // the level sums before the DMA: that frees the accumulators, which at 8
    // levels the register file needs
    double cp0[16], cp1[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      cp0[v] = (double)acc0[S - 1][v];
      cp1[v] = (double)acc1[S - 1][v];
#pragma unroll
      for (int a = S - 2; a >= 0; --a) {
        cp0[v] = fma(cp0[v], 0x1p-8, (double)acc0[a][v]);
        cp1[v] = fma(cp1[v], 0x1p-8, (double)acc1[a][v]);
      }
      // taken here: the compiler would otherwise sink some of the sums past
      // the DMA, keeping (and spilling) their accumulators
      asm volatile("" ::"v"(cp0[v]), "v"(cp1[v]));
    }
    // the exponents have landed before the DMA is issued (vmcnt(0), an
    // S_WAITCNT the compiler sees), so that no wait for them after it can
    // hold the DMA too
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __builtin_amdgcn_sched_barrier(0);
    // every wave's reads of the ring have retired, and no DMA of this item is
    // outstanding
    ring_barrier();
    const int nidx = __builtin_amdgcn_readfirstlane(item_index(slot + slots));
    WorkItem nt = it;
    if (nidx >= 0) {
      nt = p.items[nidx];
      set_dma_offsets(nt);
#pragma unroll
      for (int st = 0; st < NS; ++st)
        if (st < nsteps) issue(st, st);
    }
    __builtin_amdgcn_sched_barrier(0);
    // Every lane issues all NSTORE writes, each one instruction (c_write):
    // lanes outside a ragged item write to their own slot of the dump area,
    // so that the count the next item's first wait allows for is exact.
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int col = wn * 64 + q * 32 + le32;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const double cp = q ? cp1[v] : cp0[v];
        const int row = erow(v);
        const double add = ldexp(cp, ea[v] + fq[q] - 12);
        const bool in = row < it.h && col < it.w;
        double* dst = in ? p.C + (int64_t)(it.r0 + row) * p.ldc + it.c0 + col : p.dump + lane_e;
        c_write(dst, add, p.zero_init);
      }
    }
    it = nt;
    idx = nidx;
    if (idx >= 0) {
      // the next item's step 0 landed; its writes above are the newest
      // NSTORE vector-memory instructions and need not have completed
      if (hi) vm_wait_steps_plus<NIHI, NS - 1, NSTORE>(min(NS - 1, nsteps - 1));
      else vm_wait_steps_plus<NILO, NS - 1, NSTORE>(min(NS - 1, nsteps - 1));
      ring_barrier();
      frag_offsets(aoff, boff);
#pragma unroll
      for (int r = 0; r < LAG; ++r) read_row(0, 0, r);
    }
  }
}

__global__ __launch_bounds__(256, 1) void slice_i8_kernel(SliceArgs p) {
  __shared__ __attribute__((aligned(1024))) uint8_t smem[kBf16Lds];
  const int s = *p.slices;
  if (s <= 0) return;                          // the FP64 kernel computes this panel
  switch (s) {
    case 1: slice_i8_items<1>(p, smem); break;
    case 2: slice_i8_items<2>(p, smem); break;
    case 3: slice_i8_items<3>(p, smem); break;
    case 4: slice_i8_items<4>(p, smem); break;
    case 5: slice_i8_items<5>(p, smem); break;
    case 6: slice_i8_items<6>(p, smem); break;
    case 7: slice_i8_items<7>(p, smem); break;
    default: slice_i8_items<8>(p, smem); break;
  }
}

// ---- self-test of the matrix-core accumulation -------------------------------
// D (32 x 32, FP32) = A (32 x k digits, row-major) x B (k x 32 digits,
// row-major) by chained 32x32x16 MFMAs with FP32 accumulation -- the
// instructions and operand layout of the slice-product kernels (lane l holds
// A[l % 32][8 (l / 32) .. + 7] and B[8 (l / 32) .. + 7][l % 32]; D item v
// of lane l is D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32]).  INT8 digits
// (FMT 2) go through 32x32x32 MFMAs with INT32 accumulation (lane l holds
// A[l % 32][16 (l / 32) .. + 15] and B[16 (l / 32) .. + 15][l % 32]), and D
// is returned converted to FP32.  One wave.
template <int FMT>
__global__ __launch_bounds__(64) void mfma_probe_kernel(const void* a, const void* b, int k,
                                                         float* out) {
  const int l = threadIdx.x, l32 = l & 31, lh = l >> 5;
  if (FMT == 2) {
    const int8_t* A = (const int8_t*)a;
    const int8_t* B = (const int8_t*)b;
    i16v iacc = {};
    for (int kc = 0; kc < k; kc += 32) {
      i4v av = {}, bv = {};
      for (int e = 0; e < 16; ++e) {
        const int kk = kc + 16 * lh + e;
        av[e >> 2] |= (int)(uint8_t)A[l32 * k + kk] << (8 * (e & 3));
        bv[e >> 2] |= (int)(uint8_t)B[kk * 32 + l32] << (8 * (e & 3));
      }
      iacc = __builtin_amdgcn_mfma_i32_32x32x32_i8(av, bv, iacc, 0, 0, 0);
    }
    for (int v = 0; v < 16; ++v) out[(8 * (v >> 2) + 4 * lh + (v & 3)) * 32 + l32] = (float)iacc[v];
    return;
  }
  f16v acc = {};
  for (int kc = 0; kc < k; kc += 16) {
    if (FMT == 0) {
      const uint16_t* A = (const uint16_t*)a;
      const uint16_t* B = (const uint16_t*)b;
      bf8v av, bv;
      for (int e = 0; e < 8; ++e) {
        const int kk = kc + 8 * lh + e;
        av[e] = __builtin_bit_cast(__bf16, A[l32 * k + kk]);
        bv[e] = __builtin_bit_cast(__bf16, B[kk * 32 + l32]);
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
    } else {
      const uint8_t* A = (const uint8_t*)a;
      const uint8_t* B = (const uint8_t*)b;
      long av = 0, bv = 0;
      for (int e = 0; e < 8; ++e) {
        const int kk = kc + 8 * lh + e;
        av |= (long)A[l32 * k + kk] << (8 * e);
        bv |= (long)B[kk * 32 + l32] << (8 * e);
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(av, bv, acc, 0, 0, 0);
    }
  }
  for (int v = 0; v < 16; ++v) out[(8 * (v >> 2) + 4 * lh + (v & 3)) * 32 + l32] = acc[v];
}

hipError_t launch_mfma_probe(int fmt, const void* a, const void* b, int k, float* out,
                             hipStream_t s) {
  if (fmt == 0)
    hipLaunchKernelGGL(mfma_probe_kernel<0>, dim3(1), dim3(64), 0, s, a, b, k, out);
  else if (fmt == 1)
    hipLaunchKernelGGL(mfma_probe_kernel<1>, dim3(1), dim3(64), 0, s, a, b, k, out);
  else
    hipLaunchKernelGGL(mfma_probe_kernel<2>, dim3(1), dim3(64), 0, s, a, b, k, out);
  return hipGetLastError();
}

// ---- launchers ----------------------------------------------------------------
hipError_t launch_split(const SplitArgs& a, hipStream_t s) {
  const dim3 grid((a.m + 63) / 64 + (a.n + 63) / 64, a.nslab);
  const int gc = (int)(((int64_t)a.m + a.n + kCombineThreads - 1) / kCombineThreads);
  hipLaunchKernelGGL(split_stats_kernel, grid, dim3(64 * kSplitWaves), 0, s, a);
  hipLaunchKernelGGL(split_combine_kernel, dim3(gc), dim3(kCombineThreads), 0, s, a);
  if (a.fmt == 0)
    hipLaunchKernelGGL(split_digits_kernel<0>, grid, dim3(64 * kSplitWaves), 0, s, a);
  else if (a.fmt == 1)
    hipLaunchKernelGGL(split_digits_kernel<1>, grid, dim3(64 * kSplitWaves), 0, s, a);
  else
    hipLaunchKernelGGL(split_digits_kernel<2>, grid, dim3(64 * kSplitWaves), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* ptr, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, ptr, n);
  return hipGetLastError();
}

hipError_t launch_slices(int fmt, const SliceArgs& a, int grid, hipStream_t s) {
  if (fmt == 0)
    hipLaunchKernelGGL(slice_bf16_kernel, dim3(grid), dim3(256), 0, s, a);
  else if (fmt == 1)
    hipLaunchKernelGGL(slice_fp8_kernel, dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(slice_i8_kernel, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace hs
