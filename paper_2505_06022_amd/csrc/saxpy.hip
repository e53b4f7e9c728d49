// SAXPY, z = a*x + y: the data-parallel kernel of the paper's first listing
// (section 2), used here to measure the achievable HBM bandwidth (12 bytes
// per element: two reads and one write).
#include "ccl_internal.h"

namespace ccl {
namespace {

constexpr int kThreads = 256;
typedef float f4 __attribute__((ext_vector_type(4)));

// One 16-byte group per thread, streaming (nontemporal) loads and stores:
// the fastest of the shapes tried on gfx950 (grid-stride loops with 1, 2
// or 4 groups per thread and 4..32 blocks per CU all came out slower).
__global__ __launch_bounds__(kThreads) void saxpy_kernel(int64_t n4, int64_t n, float a,
                                                         const f4 *__restrict__ x,
                                                         const f4 *__restrict__ y,
                                                         f4 *__restrict__ z) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (i < n4) {
    const f4 xv = __builtin_nontemporal_load(&x[i]);
    const f4 yv = __builtin_nontemporal_load(&y[i]);
    f4 r;
    r.x = fmaf(a, xv.x, yv.x);
    r.y = fmaf(a, xv.y, yv.y);
    r.z = fmaf(a, xv.z, yv.z);
    r.w = fmaf(a, xv.w, yv.w);
    __builtin_nontemporal_store(r, &z[i]);
  }
  // scalar tail (fewer than 4 elements), handled by the first threads
  const int64_t k = n4 * 4 + i;
  if (k < n) {
    const float *xs = reinterpret_cast<const float *>(x);
    const float *ys = reinterpret_cast<const float *>(y);
    float *zs = reinterpret_cast<float *>(z);
    zs[k] = fmaf(a, xs[k], ys[k]);
  }
}

}  // namespace
}  // namespace ccl

using namespace ccl;

extern "C" ccl_status ccl_saxpy(int64_t n, float a, const float *x, const float *y, float *z,
                                void *hip_stream) {
  clear_error();
  if (n < 0) return fail(CCL_E_INVALID, "n=%lld < 0", (long long)n);
  if (n == 0) return CCL_OK;
  if (!x || !y || !z) return fail(CCL_E_INVALID, "NULL argument");
  if (((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y) |
        reinterpret_cast<uintptr_t>(z)) & 15u) != 0)
    return fail(CCL_E_INVALID, "x, y, z must be 16-byte aligned");
  const int64_t n4 = n / 4;
  int64_t blocks = (n4 + kThreads - 1) / kThreads;
  if (blocks < 1) blocks = 1;
  if (blocks > INT32_MAX) return fail(CCL_E_RANGE, "n too large for one launch");
  TimedLaunch tl(CCL_KERNEL_SAXPY, static_cast<hipStream_t>(hip_stream));
  hipLaunchKernelGGL(saxpy_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kThreads), 0,
                     static_cast<hipStream_t>(hip_stream), n4, n, a,
                     reinterpret_cast<const f4 *>(x), reinterpret_cast<const f4 *>(y),
                     reinterpret_cast<f4 *>(z));
  return hip_check(hipGetLastError(), "saxpy_kernel launch");
}
