// Cost-model network kernels (the learned form of the tuner): a 3-layer
// FP32 MLP  Z = W3^T relu(W2^T relu(W1^T x + b1) + b2) + b3  that predicts
// the log run time of every candidate kernel configuration of one problem
// shape, trained on the tuner's own timings with a masked mean squared
// error and Adam.  Every step of training and inference runs here.
//
// Parameter block (floats, contiguous): W1 (F x H), b1 (H), W2 (H x H),
// b2 (H), W3 (H x K), b3 (K), all row-major.  Work block: A1, A2 (N x H
// pre-activations), H1, H2 (N x H activations), dZ (N x K), dA1, dA2
// (N x H).  The network is tiny (H = 64); the kernels are plain
// one-thread-per-output loops, sized for clarity rather than speed.
#include "internal.h"

namespace hs {

struct MlpDims {
  int N, F, H, K;
};

__host__ __device__ inline int64_t mlp_param_count(int F, int H, int K) {
  return (int64_t)F * H + H + (int64_t)H * H + H + (int64_t)H * K + K;
}

// Y (N x J) = act(X (N x I) W (I x J) + b); pre-activation kept in Apre.
__global__ void mlp_linear_fwd(const float* __restrict__ X, const float* __restrict__ W,
                               const float* __restrict__ b, float* __restrict__ Apre,
                               float* __restrict__ Y, int N, int I, int J, int relu) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)N * J) return;
  const int i = (int)(t / J), j = (int)(t % J);
  float acc = b[j];
  for (int k = 0; k < I; ++k) acc = fmaf(X[(int64_t)i * I + k], W[(int64_t)k * J + j], acc);
  if (Apre) Apre[t] = acc;
  Y[t] = relu ? fmaxf(acc, 0.0f) : acc;
}

// dZ = 2 mask (Z - T) / max(1, sum(mask)); loss = sum(mask (Z - T)^2) / ...
// One block; the mask count and the loss are block reductions.
__global__ void mlp_mse_grad(const float* __restrict__ Z, const float* __restrict__ T,
                             const float* __restrict__ mask, float* __restrict__ dZ,
                             float* __restrict__ loss, int64_t n) {
  __shared__ float s_cnt[256], s_sum[256];
  float cnt = 0.f, sum = 0.f;
  for (int64_t t = threadIdx.x; t < n; t += blockDim.x) {
    const float d = (Z[t] - T[t]) * mask[t];
    cnt += mask[t];
    sum += d * d;
  }
  s_cnt[threadIdx.x] = cnt;
  s_sum[threadIdx.x] = sum;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s_cnt[threadIdx.x] += s_cnt[threadIdx.x + o];
      s_sum[threadIdx.x] += s_sum[threadIdx.x + o];
    }
    __syncthreads();
  }
  const float c = fmaxf(1.0f, s_cnt[0]);
  if (threadIdx.x == 0 && loss) *loss = s_sum[0] / c;
  for (int64_t t = threadIdx.x; t < n; t += blockDim.x) dZ[t] = 2.0f * (Z[t] - T[t]) * mask[t] / c;
}

// dW (I x J) = X^T dY,  X: N x I, dY: N x J
__global__ void mlp_grad_w(const float* __restrict__ X, const float* __restrict__ dY,
                           float* __restrict__ dW, int N, int I, int J) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)I * J) return;
  const int k = (int)(t / J), j = (int)(t % J);
  float acc = 0.f;
  for (int i = 0; i < N; ++i) acc = fmaf(X[(int64_t)i * I + k], dY[(int64_t)i * J + j], acc);
  dW[t] = acc;
}

// db (J) = sum over rows of dY
__global__ void mlp_grad_b(const float* __restrict__ dY, float* __restrict__ db, int N, int J) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= J) return;
  float acc = 0.f;
  for (int i = 0; i < N; ++i) acc += dY[(int64_t)i * J + j];
  db[j] = acc;
}

// dA (N x I) = (dY W^T) * (Apre > 0),  W: I x J
__global__ void mlp_grad_x_relu(const float* __restrict__ dY, const float* __restrict__ W,
                                const float* __restrict__ Apre, float* __restrict__ dA, int N,
                                int I, int J) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)N * I) return;
  const int i = (int)(t / I), k = (int)(t % I);
  float acc = 0.f;
  for (int j = 0; j < J; ++j) acc = fmaf(dY[(int64_t)i * J + j], W[(int64_t)k * J + j], acc);
  dA[t] = Apre[t] > 0.f ? acc : 0.f;
}

// Adam with bias correction (Kingma and Ba, 2015), in place.
__global__ void mlp_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                         float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                         float c1, float c2) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float gt = g[t];
  const float mt = b1 * m[t] + (1.f - b1) * gt;
  const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
  m[t] = mt;
  v[t] = vt;
  p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

static inline unsigned blocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

struct MlpPtrs {
  const float *W1, *b1, *W2, *b2, *W3, *b3;
};
static MlpPtrs unpack(const float* P, int F, int H, int K) {
  MlpPtrs q;
  q.W1 = P;
  q.b1 = q.W1 + (int64_t)F * H;
  q.W2 = q.b1 + H;
  q.b2 = q.W2 + (int64_t)H * H;
  q.W3 = q.b2 + H;
  q.b3 = q.W3 + (int64_t)H * K;
  return q;
}

hipError_t mlp_forward(const MlpDims& d, const float* X, const float* P, float* Z, float* work,
                       hipStream_t s) {
  const MlpPtrs q = unpack(P, d.F, d.H, d.K);
  float* A1 = work;
  float* A2 = A1 + (int64_t)d.N * d.H;
  float* H1 = A2 + (int64_t)d.N * d.H;
  float* H2 = H1 + (int64_t)d.N * d.H;
  const int bs = 256;
  hipLaunchKernelGGL(mlp_linear_fwd, dim3(blocks((int64_t)d.N * d.H, bs)), dim3(bs), 0, s, X, q.W1,
                     q.b1, A1, H1, d.N, d.F, d.H, 1);
  hipLaunchKernelGGL(mlp_linear_fwd, dim3(blocks((int64_t)d.N * d.H, bs)), dim3(bs), 0, s, H1, q.W2,
                     q.b2, A2, H2, d.N, d.H, d.H, 1);
  hipLaunchKernelGGL(mlp_linear_fwd, dim3(blocks((int64_t)d.N * d.K, bs)), dim3(bs), 0, s, H2, q.W3,
                     q.b3, (float*)nullptr, Z, d.N, d.H, d.K, 0);
  return hipGetLastError();
}

hipError_t mlp_grad(const MlpDims& d, const float* X, const float* T, const float* mask,
                    const float* P, float* G, float* Z, float* loss, float* work, hipStream_t s) {
  hipError_t e = mlp_forward(d, X, P, Z, work, s);
  if (e != hipSuccess) return e;
  const MlpPtrs q = unpack(P, d.F, d.H, d.K);
  float* gW1 = G;
  float* gb1 = gW1 + (int64_t)d.F * d.H;
  float* gW2 = gb1 + d.H;
  float* gb2 = gW2 + (int64_t)d.H * d.H;
  float* gW3 = gb2 + d.H;
  float* gb3 = gW3 + (int64_t)d.H * d.K;
  const int64_t NH = (int64_t)d.N * d.H;
  float* A1 = work;
  float* A2 = A1 + NH;
  float* H1 = A2 + NH;
  float* H2 = H1 + NH;
  float* dZ = H2 + NH;
  float* dA2 = dZ + (int64_t)d.N * d.K;
  float* dA1 = dA2 + NH;
  const int bs = 256;
  hipLaunchKernelGGL(mlp_mse_grad, dim3(1), dim3(256), 0, s, Z, T, mask, dZ, loss,
                     (int64_t)d.N * d.K);
  hipLaunchKernelGGL(mlp_grad_w, dim3(blocks((int64_t)d.H * d.K, bs)), dim3(bs), 0, s, H2, dZ, gW3,
                     d.N, d.H, d.K);
  hipLaunchKernelGGL(mlp_grad_b, dim3(blocks(d.K, bs)), dim3(bs), 0, s, dZ, gb3, d.N, d.K);
  hipLaunchKernelGGL(mlp_grad_x_relu, dim3(blocks(NH, bs)), dim3(bs), 0, s, dZ, q.W3, A2, dA2, d.N,
                     d.H, d.K);
  hipLaunchKernelGGL(mlp_grad_w, dim3(blocks((int64_t)d.H * d.H, bs)), dim3(bs), 0, s, H1, dA2, gW2,
                     d.N, d.H, d.H);
  hipLaunchKernelGGL(mlp_grad_b, dim3(blocks(d.H, bs)), dim3(bs), 0, s, dA2, gb2, d.N, d.H);
  hipLaunchKernelGGL(mlp_grad_x_relu, dim3(blocks(NH, bs)), dim3(bs), 0, s, dA2, q.W2, A1, dA1, d.N,
                     d.H, d.H);
  hipLaunchKernelGGL(mlp_grad_w, dim3(blocks((int64_t)d.F * d.H, bs)), dim3(bs), 0, s, X, dA1, gW1,
                     d.N, d.F, d.H);
  hipLaunchKernelGGL(mlp_grad_b, dim3(blocks(d.H, bs)), dim3(bs), 0, s, dA1, gb1, d.N, d.H);
  return hipGetLastError();
}

hipError_t mlp_adam_step(float* P, const float* G, float* M, float* V, int64_t n, float lr,
                         float b1, float b2, float eps, int t, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(mlp_adam, dim3(blocks(n, 256)), dim3(256), 0, s, P, G, M, V, n, lr, b1, b2,
                     eps, c1, c2);
  return hipGetLastError();
}

}  // namespace hs

// ---- C ABI --------------------------------------------------------------------
extern "C" {

int64_t hsumma_mlp_param_count(int32_t F, int32_t H, int32_t K) {
  if (F < 1 || H < 1 || K < 1) return -1;
  return hs::mlp_param_count(F, H, K);
}

int64_t hsumma_mlp_work_floats(int32_t N, int32_t H, int32_t K) {
  if (N < 1 || H < 1 || K < 1) return -1;
  return 6 * (int64_t)N * H + (int64_t)N * K;
}

static int mlp_check(int32_t N, int32_t F, int32_t H, int32_t K) {
  if (N < 1 || F < 1 || H < 1 || K < 1 || (int64_t)N * (H > K ? H : K) >= (1LL << 31)) {
    hs::set_error("MLP dimensions must be positive (and N x max(H, K) < 2^31)");
    return HSUMMA_ERR_INVALID;
  }
  return HSUMMA_OK;
}

int hsumma_mlp_forward(int32_t N, int32_t F, int32_t H, int32_t K, const float* X,
                       const float* params, float* Z, float* work, void* stream) {
  int rc = mlp_check(N, F, H, K);
  if (rc) return rc;
  if (!X || !params || !Z || !work) {
    hs::set_error("null pointer");
    return HSUMMA_ERR_INVALID;
  }
  hipError_t e = hs::mlp_forward(hs::MlpDims{N, F, H, K}, X, params, Z, work, (hipStream_t)stream);
  if (e != hipSuccess) {
    hs::set_error(std::string("mlp forward: ") + hipGetErrorString(e));
    return HSUMMA_ERR_DEVICE;
  }
  return HSUMMA_OK;
}

int hsumma_mlp_grad(int32_t N, int32_t F, int32_t H, int32_t K, const float* X, const float* T,
                    const float* mask, const float* params, float* grads, float* Z, float* loss,
                    float* work, void* stream) {
  int rc = mlp_check(N, F, H, K);
  if (rc) return rc;
  if (!X || !T || !mask || !params || !grads || !Z || !work) {
    hs::set_error("null pointer");
    return HSUMMA_ERR_INVALID;
  }
  hipError_t e = hs::mlp_grad(hs::MlpDims{N, F, H, K}, X, T, mask, params, grads, Z, loss, work,
                              (hipStream_t)stream);
  if (e != hipSuccess) {
    hs::set_error(std::string("mlp grad: ") + hipGetErrorString(e));
    return HSUMMA_ERR_DEVICE;
  }
  return HSUMMA_OK;
}

int hsumma_mlp_adam(int64_t n, float* params, const float* grads, float* m, float* v, float lr,
                    float beta1, float beta2, float eps, int32_t step, void* stream) {
  if (n < 1 || !params || !grads || !m || !v || step < 1) {
    hs::set_error("bad Adam arguments");
    return HSUMMA_ERR_INVALID;
  }
  hipError_t e = hs::mlp_adam_step(params, grads, m, v, n, lr, beta1, beta2, eps, step,
                                   (hipStream_t)stream);
  if (e != hipSuccess) {
    hs::set_error(std::string("mlp adam: ") + hipGetErrorString(e));
    return HSUMMA_ERR_DEVICE;
  }
  return HSUMMA_OK;
}

}  // extern "C"
