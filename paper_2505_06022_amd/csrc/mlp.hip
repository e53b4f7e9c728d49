// The launch-config cost model: a 12-64-64-2 float32 MLP with ReLU, trained
// on the GPU with mean-squared error and Adam (Kingma & Ba, 2015), and a
// pick kernel that scores every candidate config of a shape and returns the
// best one.
//
// Parameters are packed W1 (64x12), b1, W2 (64x64), b2, W3 (2x64), b3, row
// major (W[out][in]).  Training is deterministic: a block handles a fixed
// slice of 64 samples and writes its partial gradient; a second kernel sums
// the partials in block order; no floating-point atomics anywhere.  Every
// dot product accumulates with fma in ascending index order.
#include <cmath>
#include <cstring>
#include <vector>

#include "ccl_internal.h"

namespace ccl {
namespace {

constexpr int kIn = CCL_MLP_IN, kHid = CCL_MLP_HIDDEN, kOut = CCL_MLP_OUT;
constexpr int oW1 = 0, ob1 = oW1 + kHid * kIn, oW2 = ob1 + kHid, ob2 = oW2 + kHid * kHid,
              oW3 = ob2 + kHid, ob3 = oW3 + kOut * kHid, kParams = ob3 + kOut;
static_assert(kParams == CCL_MLP_NPARAMS, "parameter count");
constexpr int kS = 64;          // samples per block in the gradient kernel
constexpr int kThreads = 256;

__device__ __forceinline__ void load_params(float *sp, const float *p) {
  for (int i = threadIdx.x; i < kParams; i += blockDim.x) sp[i] = p[i];
}

// Partial gradient of L = 1/(2n) sum w (y - t)^2 over this block's samples
// (w = 1 where no weights are given).
__global__ __launch_bounds__(kThreads) void mlp_grad_kernel(const float *__restrict__ params,
                                                            const float *__restrict__ x,
                                                            const float *__restrict__ t,
                                                            const float *__restrict__ w, int n,
                                                            float *__restrict__ partials,
                                                            float *__restrict__ loss_partials) {
  __shared__ float P[kParams];
  __shared__ float X[kS][kIn];
  __shared__ float H1[kS][kHid];
  __shared__ float H2[kS][kHid];
  __shared__ float DY[kS][kOut];
  __shared__ float WR[kS][kOut];
  // H2 and H1 are overwritten in place by the back-propagated D2 and D1
  // once every reader of the activations is done (56 KB of LDS in all).
  float(*D2)[kHid] = H2;
  float(*D1)[kHid] = H1;
  const int tid = threadIdx.x;
  const int s0 = blockIdx.x * kS;
  const int ns = min(kS, n - s0);
  const float inv_n = 1.0f / static_cast<float>(n);
  load_params(P, params);
  for (int i = tid; i < kS * kIn; i += kThreads) {
    const int s = i / kIn, k = i - s * kIn;
    X[s][k] = s < ns ? x[static_cast<int64_t>(s0 + s) * kIn + k] : 0.0f;
  }
  __syncthreads();
  // forward
  for (int i = tid; i < kS * kHid; i += kThreads) {
    const int s = i / kHid, j = i - s * kHid;
    float acc = P[ob1 + j];
    for (int k = 0; k < kIn; ++k) acc = fmaf(P[oW1 + j * kIn + k], X[s][k], acc);
    H1[s][j] = acc > 0.0f ? acc : 0.0f;
  }
  __syncthreads();
  for (int i = tid; i < kS * kHid; i += kThreads) {
    const int s = i / kHid, j = i - s * kHid;
    float acc = P[ob2 + j];
    for (int k = 0; k < kHid; ++k) acc = fmaf(P[oW2 + j * kHid + k], H1[s][k], acc);
    H2[s][j] = acc > 0.0f ? acc : 0.0f;
  }
  __syncthreads();
  if (tid < kS * kOut) {
    const int s = tid / kOut, o = tid - s * kOut;
    float acc = P[ob3 + o];
    for (int k = 0; k < kHid; ++k) acc = fmaf(P[oW3 + o * kHid + k], H2[s][k], acc);
    const int64_t q = static_cast<int64_t>(s0 + s) * kOut + o;
    const float r = s < ns ? acc - t[q] : 0.0f;
    const float wt = (s < ns && w) ? w[q] : 1.0f;
    DY[s][o] = r * wt;        // w * residual; scaled by 1/n below
    WR[s][o] = r;
  }
  __syncthreads();
  if (tid == 0) {
    float l = 0.0f;
    for (int s = 0; s < ns; ++s)
      for (int o = 0; o < kOut; ++o) l = fmaf(DY[s][o], WR[s][o], l);
    loss_partials[blockIdx.x] = l;
  }
  __syncthreads();
  if (tid < kS * kOut) {
    const int s = tid / kOut, o = tid - s * kOut;
    DY[s][o] *= inv_n;
  }
  __syncthreads();
  float *out = partials + static_cast<int64_t>(blockIdx.x) * kParams;
  // layer 3
  for (int i = tid; i < kOut * kHid; i += kThreads) {
    const int o = i / kHid, k = i - o * kHid;
    float acc = 0.0f;
    for (int s = 0; s < kS; ++s) acc = fmaf(DY[s][o], H2[s][k], acc);
    out[oW3 + i] = acc;
  }
  if (tid < kOut) {
    float acc = 0.0f;
    for (int s = 0; s < kS; ++s) acc += DY[s][tid];
    out[ob3 + tid] = acc;
  }
  __syncthreads();  // H2 read by dW3 above; D2 replaces it below
  for (int i = tid; i < kS * kHid; i += kThreads) {
    const int s = i / kHid, k = i - s * kHid;
    float acc = 0.0f;
    for (int o = 0; o < kOut; ++o) acc = fmaf(DY[s][o], P[oW3 + o * kHid + k], acc);
    D2[s][k] = H2[s][k] > 0.0f ? acc : 0.0f;
  }
  __syncthreads();
  // layer 2
  for (int i = tid; i < kHid * kHid; i += kThreads) {
    const int j = i / kHid, k = i - j * kHid;
    float acc = 0.0f;
    for (int s = 0; s < kS; ++s) acc = fmaf(D2[s][j], H1[s][k], acc);
    out[oW2 + i] = acc;
  }
  if (tid < kHid) {
    float acc = 0.0f;
    for (int s = 0; s < kS; ++s) acc += D2[s][tid];
    out[ob2 + tid] = acc;
  }
  __syncthreads();  // H1 read by dW2 above; D1 replaces it below
  for (int i = tid; i < kS * kHid; i += kThreads) {
    const int s = i / kHid, k = i - s * kHid;
    float acc = 0.0f;
    for (int j = 0; j < kHid; ++j) acc = fmaf(D2[s][j], P[oW2 + j * kHid + k], acc);
    D1[s][k] = H1[s][k] > 0.0f ? acc : 0.0f;
  }
  __syncthreads();
  // layer 1
  for (int i = tid; i < kHid * kIn; i += kThreads) {
    const int j = i / kIn, k = i - j * kIn;
    float acc = 0.0f;
    for (int s = 0; s < kS; ++s) acc = fmaf(D1[s][j], X[s][k], acc);
    out[oW1 + i] = acc;
  }
  if (tid < kHid) {
    float acc = 0.0f;
    for (int s = 0; s < kS; ++s) acc += D1[s][tid];
    out[ob1 + tid] = acc;
  }
}

// grads[p] = sum over blocks (in block order) of partials[b][p]; loss too.
__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float *__restrict__ partials,
                                                         const float *__restrict__ loss_partials,
                                                         int nblocks, int n,
                                                         float *__restrict__ grads,
                                                         float *__restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kParams) {
    float acc = 0.0f;
    for (int b = 0; b < nblocks; ++b) acc += partials[static_cast<int64_t>(b) * kParams + p];
    grads[p] = acc;
  }
  if (p == 0) {
    float l = 0.0f;
    for (int b = 0; b < nblocks; ++b) l += loss_partials[b];
    *loss = 0.5f * l / static_cast<float>(n);
  }
}

__global__ __launch_bounds__(256) void mlp_adam_kernel(float *__restrict__ params,
                                                       const float *__restrict__ grads,
                                                       float *__restrict__ m,
                                                       float *__restrict__ v, float lr, float b1,
                                                       float b2, float eps, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  const float g = grads[p];
  const float mm = fmaf(b1, m[p], (1.0f - b1) * g);
  const float vv = fmaf(b2, v[p], (1.0f - b2) * g * g);
  m[p] = mm;
  v[p] = vv;
  const float mhat = mm * c1;
  const float vhat = vv * c2;
  params[p] -= lr * mhat / (sqrtf(vhat) + eps);
}

// y = net(x) for n samples, one sample per thread.
__device__ __forceinline__ void forward_one(const float *P, const float *xs, float *y) {
  float h1[kHid];
  for (int j = 0; j < kHid; ++j) {
    float acc = P[ob1 + j];
    for (int k = 0; k < kIn; ++k) acc = fmaf(P[oW1 + j * kIn + k], xs[k], acc);
    h1[j] = acc > 0.0f ? acc : 0.0f;
  }
  float y0 = P[ob3 + 0], y1 = P[ob3 + 1];
  for (int j = 0; j < kHid; ++j) {
    float acc = P[ob2 + j];
    for (int k = 0; k < kHid; ++k) acc = fmaf(P[oW2 + j * kHid + k], h1[k], acc);
    const float h2 = acc > 0.0f ? acc : 0.0f;
    y0 = fmaf(P[oW3 + j], h2, y0);
    y1 = fmaf(P[oW3 + kHid + j], h2, y1);
  }
  y[0] = y0;
  y[1] = y1;
}

__global__ __launch_bounds__(256) void mlp_forward_kernel(const float *__restrict__ params,
                                                          const float *__restrict__ x, int n,
                                                          float *__restrict__ y) {
  __shared__ float P[kParams];
  load_params(P, params);
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float xs[kIn];
  for (int k = 0; k < kIn; ++k) xs[k] = x[static_cast<int64_t>(i) * kIn + k];
  float out[kOut];
  forward_one(P, xs, out);
  y[static_cast<int64_t>(i) * kOut + 0] = out[0];
  y[static_cast<int64_t>(i) * kOut + 1] = out[1];
}

constexpr int kMaxRank = 4096;

// One block: the score of every candidate (as mlp_pick_kernel computes it)
// kept in LDS, then k rounds of a block argmin (ties: the lowest index),
// each removing its winner: the k best in ascending order.  k <= n, so every
// round finds a candidate (scores of +inf included).
__global__ __launch_bounds__(256) void mlp_rank_kernel(const float *__restrict__ params,
                                                       const float *__restrict__ x, int n,
                                                       float w0, float w1, int k,
                                                       int32_t *__restrict__ order) {
  __shared__ float P[kParams];
  __shared__ float sc[kMaxRank];
  __shared__ float bs[256];
  __shared__ int bi[256];
  load_params(P, params);
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    float xs[kIn];
    for (int q = 0; q < kIn; ++q) xs[q] = x[static_cast<int64_t>(i) * kIn + q];
    float out[kOut];
    forward_one(P, xs, out);
    const float s = fmaf(w1, out[1], w0 * out[0]);
    sc[i] = s == s ? s : INFINITY;  // a NaN score ranks with +inf (lowest index first)
  }
  __syncthreads();
  for (int r = 0; r < k; ++r) {
    float my_s = INFINITY;
    int my_i = INT32_MAX;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const float s = sc[i];
      if (s < my_s || (s == my_s && i < my_i)) {
        my_s = s;
        my_i = i;
      }
    }
    bs[threadIdx.x] = my_s;
    bi[threadIdx.x] = my_i;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) {
        const float os = bs[threadIdx.x + w];
        const int oi = bi[threadIdx.x + w];
        if (os < bs[threadIdx.x] || (os == bs[threadIdx.x] && oi < bi[threadIdx.x])) {
          bs[threadIdx.x] = os;
          bi[threadIdx.x] = oi;
        }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      order[r] = bi[0];
      sc[bi[0]] = NAN;  // removed: no comparison selects a NaN
    }
    __syncthreads();
  }
}

// One block: score_i = w0*y_i0 + w1*y_i1 for every candidate, then the index
// of the smallest score (ties: the lowest index).
__global__ __launch_bounds__(256) void mlp_pick_kernel(const float *__restrict__ params,
                                                       const float *__restrict__ x, int n,
                                                       float w0, float w1,
                                                       float *__restrict__ scores,
                                                       int32_t *__restrict__ best) {
  __shared__ float P[kParams];
  __shared__ float bs[256];
  __shared__ int bi[256];
  load_params(P, params);
  __syncthreads();
  float my_s = INFINITY;
  int my_i = INT32_MAX;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    float xs[kIn];
    for (int k = 0; k < kIn; ++k) xs[k] = x[static_cast<int64_t>(i) * kIn + k];
    float out[kOut];
    forward_one(P, xs, out);
    const float s = fmaf(w1, out[1], w0 * out[0]);
    if (scores) scores[i] = s;
    if (s < my_s || (s == my_s && i < my_i)) {
      my_s = s;
      my_i = i;
    }
  }
  bs[threadIdx.x] = my_s;
  bi[threadIdx.x] = my_i;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const float os = bs[threadIdx.x + w];
      const int oi = bi[threadIdx.x + w];
      if (os < bs[threadIdx.x] || (os == bs[threadIdx.x] && oi < bi[threadIdx.x])) {
        bs[threadIdx.x] = os;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *best = bi[0];
}

}  // namespace
}  // namespace ccl

using namespace ccl;

struct ccl_mlp {
  float *dev = nullptr;  // params | grads | m | v | loss | partials...
  float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr, *loss = nullptr;
  float *partials = nullptr, *loss_partials = nullptr;
  int32_t max_blocks = 0;
  int64_t step = 0;  // Adam steps taken
};

static ccl_status mlp_reserve(ccl_mlp *M, int32_t n) {
  const int32_t blocks = (n + kS - 1) / kS;
  if (blocks <= M->max_blocks) return CCL_OK;
  if (M->partials) (void)hipFree(M->partials);
  M->partials = nullptr;
  M->max_blocks = 0;
  const size_t bytes = (static_cast<size_t>(blocks) * kParams + blocks) * sizeof(float);
  ccl_status st = hip_check(hipMalloc(&M->partials, bytes), "hipMalloc(mlp partials)");
  if (st != CCL_OK) return st;
  M->loss_partials = M->partials + static_cast<size_t>(blocks) * kParams;
  M->max_blocks = blocks;
  return CCL_OK;
}

extern "C" ccl_status ccl_mlp_create(const float *params, ccl_mlp **out) {
  clear_error();
  if (!params || !out) return fail(CCL_E_INVALID, "NULL argument");
  for (int i = 0; i < kParams; ++i)
    if (!std::isfinite(params[i])) return fail(CCL_E_INVALID, "parameter %d is not finite", i);
  ccl_mlp *M = new ccl_mlp();
  const size_t words = 4 * static_cast<size_t>(kParams) + 64;
  ccl_status st = hip_check(hipMalloc(&M->dev, words * sizeof(float)), "hipMalloc(mlp)");
  if (st != CCL_OK) {
    delete M;
    return st;
  }
  M->params = M->dev;
  M->grads = M->params + kParams;
  M->m = M->grads + kParams;
  M->v = M->m + kParams;
  M->loss = M->v + kParams;
  hipError_t e = hipMemcpy(M->params, params, kParams * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(M->grads, 0, (3 * static_cast<size_t>(kParams) + 64) * sizeof(float));
  if (e != hipSuccess) {
    (void)hipFree(M->dev);
    delete M;
    return hip_check(e, "mlp init");
  }
  *out = M;
  return CCL_OK;
}

extern "C" ccl_status ccl_mlp_destroy(ccl_mlp *M) {
  clear_error();
  if (!M) return CCL_OK;
  if (M->partials) (void)hipFree(M->partials);
  if (M->dev) (void)hipFree(M->dev);
  delete M;
  return CCL_OK;
}

extern "C" ccl_status ccl_mlp_get(const ccl_mlp *M, int32_t what, float *host_out) {
  clear_error();
  if (!M || !host_out) return fail(CCL_E_INVALID, "NULL argument");
  const float *src = what == CCL_MLP_PARAMS ? M->params
                     : what == CCL_MLP_GRADS ? M->grads
                     : what == CCL_MLP_LOSS  ? M->loss
                                             : nullptr;
  if (!src) return fail(CCL_E_INVALID, "unknown quantity %d", what);
  const size_t n = what == CCL_MLP_LOSS ? 1 : kParams;
  return hip_check(hipMemcpy(host_out, src, n * sizeof(float), hipMemcpyDeviceToHost),
                   "hipMemcpy(mlp get)");
}

extern "C" ccl_status ccl_mlp_forward(ccl_mlp *M, int32_t n, const float *x, float *y,
                                      void *hip_stream) {
  clear_error();
  if (!M || n < 0 || (n > 0 && (!x || !y))) return fail(CCL_E_INVALID, "bad argument");
  if (n == 0) return CCL_OK;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((n + 255) / 256), dim3(256), 0,
                     static_cast<hipStream_t>(hip_stream), M->params, x, n, y);
  return hip_check(hipGetLastError(), "mlp_forward_kernel launch");
}

extern "C" ccl_status ccl_mlp_grad_weighted(ccl_mlp *M, int32_t n, const float *x,
                                            const float *t, const float *w, void *hip_stream) {
  clear_error();
  if (!M || n < 1 || !x || !t) return fail(CCL_E_INVALID, "bad argument");
  ccl_status st = mlp_reserve(M, n);
  if (st != CCL_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int blocks = (n + kS - 1) / kS;
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(blocks), dim3(kThreads), 0, s, M->params, x, t, w, n,
                     M->partials, M->loss_partials);
  st = hip_check(hipGetLastError(), "mlp_grad_kernel launch");
  if (st != CCL_OK) return st;
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s,
                     M->partials, M->loss_partials, blocks, n, M->grads, M->loss);
  return hip_check(hipGetLastError(), "mlp_reduce_kernel launch");
}

extern "C" ccl_status ccl_mlp_grad(ccl_mlp *M, int32_t n, const float *x, const float *t,
                                   void *hip_stream) {
  return ccl_mlp_grad_weighted(M, n, x, t, nullptr, hip_stream);
}

extern "C" ccl_status ccl_mlp_adam(ccl_mlp *M, float lr, float b1, float b2, float eps,
                                   void *hip_stream) {
  clear_error();
  if (!M) return fail(CCL_E_INVALID, "NULL model");
  if (!(lr > 0.0f) || !(b1 >= 0.0f && b1 < 1.0f) || !(b2 >= 0.0f && b2 < 1.0f) || !(eps > 0.0f))
    return fail(CCL_E_INVALID, "bad Adam hyper-parameters");
  M->step += 1;
  const double c1 = 1.0 / (1.0 - std::pow(static_cast<double>(b1), static_cast<double>(M->step)));
  const double c2 = 1.0 / (1.0 - std::pow(static_cast<double>(b2), static_cast<double>(M->step)));
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((kParams + 255) / 256), dim3(256), 0,
                     static_cast<hipStream_t>(hip_stream), M->params, M->grads, M->m, M->v, lr,
                     b1, b2, eps, static_cast<float>(c1), static_cast<float>(c2));
  return hip_check(hipGetLastError(), "mlp_adam_kernel launch");
}

extern "C" ccl_status ccl_mlp_train(ccl_mlp *M, int32_t n, const float *x, const float *t,
                                    const float *w, int32_t epochs, float lr,
                                    void *hip_stream) {
  clear_error();
  if (!M || epochs < 0) return fail(CCL_E_INVALID, "bad argument");
  for (int e = 0; e < epochs; ++e) {
    ccl_status st = ccl_mlp_grad_weighted(M, n, x, t, w, hip_stream);
    if (st != CCL_OK) return st;
    st = ccl_mlp_adam(M, lr, 0.9f, 0.999f, 1e-8f, hip_stream);
    if (st != CCL_OK) return st;
  }
  return CCL_OK;
}

extern "C" ccl_status ccl_mlp_rank(ccl_mlp *M, int32_t n, const float *x, float w_time,
                                   float w_energy, int32_t k, int32_t *order,
                                   void *hip_stream) {
  clear_error();
  if (!M || n < 1 || !x || !order || k < 1 || k > n) return fail(CCL_E_INVALID, "bad argument");
  if (n > kMaxRank) return fail(CCL_E_RANGE, "n=%d above %d", n, kMaxRank);
  hipLaunchKernelGGL(mlp_rank_kernel, dim3(1), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                     M->params, x, n, w_time, w_energy, k, order);
  return hip_check(hipGetLastError(), "mlp_rank_kernel launch");
}

extern "C" ccl_status ccl_mlp_pick(ccl_mlp *M, int32_t n, const float *x, float w_time,
                                   float w_energy, float *scores, int32_t *best,
                                   void *hip_stream) {
  clear_error();
  if (!M || n < 1 || !x || !best) return fail(CCL_E_INVALID, "bad argument");
  hipLaunchKernelGGL(mlp_pick_kernel, dim3(1), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                     M->params, x, n, w_time, w_energy, scores, best);
  return hip_check(hipGetLastError(), "mlp_pick_kernel launch");
}
