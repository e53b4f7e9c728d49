// Discrete energy of the leapfrog scheme on the device, for monitoring a
// run's conservation without copying its fields to the host:
//   E^{n+1/2} = sum_i (a_i - b_i)^2 + r2 * sum_{edges (p,q)} (a_p - a_q)(b_p - b_q)
// with a = u^{n+1}, b = u^n, over every edge of the grid, those to the zero
// cells just outside the domain included.  Each edge is taken once: from a
// cell to its successor along each dimension (a zero cell past the last
// one), plus, for cells at index 0 of a dimension, the edge from the zero
// cell before them, whose term is a_i * b_i.
//
// Work unit: a block streams whole rows (grid-stride over rows, threads
// strided along the row); per-cell terms are formed in double from the
// exactly widened inputs and summed in double per thread, then per block in
// a fixed order; a second one-block kernel sums the per-block partials in a
// fixed order, so the result is deterministic for a given shape.  Bound:
// HBM (each element read once from memory; the +y / +z neighbours are the
// rows the block or its neighbours read, served by L2).
#include <algorithm>

#include "ccl_internal.h"
#include "prec.h"

namespace ccl {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 1024;

struct EnergyArgs {
  const void *a;  // u^{n+1}
  const void *b;  // u^n
  int64_t nz, ny, nx;  // nz = 1 in 2D
  int64_t pz, py;      // element strides of planes and rows
  int32_t zdim;        // 1 if the field has a z dimension (3D)
  double r2;
  double *partial;     // one per block
};

template <class PR>
__device__ __forceinline__ double at(const void *base, int64_t off) {
  return static_cast<double>(PR::widen(static_cast<const typename PR::E *>(base)[off]));
}

// Sum of a block's per-thread values in a fixed order: within each wave a
// shuffle tree (lane 0 ends with the wave's sum), then the waves' sums in
// index order; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *lds) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kThreads / 64; ++w) s += lds[w];
  return s;
}

template <class PR>
__global__ __launch_bounds__(kThreads) void energy_kernel(const EnergyArgs g) {
  __shared__ double lds[kThreads / 64];
  const int64_t rows = g.nz * g.ny;
  double acc = 0.0;
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const int64_t z = r / g.ny, y = r - z * g.ny;
    const int64_t row = z * g.pz + y * g.py;
    const bool yl = y + 1 < g.ny, zl = g.zdim && z + 1 < g.nz;
    for (int64_t x = threadIdx.x; x < g.nx; x += kThreads) {
      const int64_t o = row + x;
      const double a = at<PR>(g.a, o), b = at<PR>(g.b, o);
      double e = 0.0;  // edge terms of this cell
      const double ax = x + 1 < g.nx ? at<PR>(g.a, o + 1) : 0.0;
      const double bx = x + 1 < g.nx ? at<PR>(g.b, o + 1) : 0.0;
      e += (a - ax) * (b - bx);
      const double ay = yl ? at<PR>(g.a, o + g.py) : 0.0;
      const double by = yl ? at<PR>(g.b, o + g.py) : 0.0;
      e += (a - ay) * (b - by);
      if (g.zdim) {
        const double az = zl ? at<PR>(g.a, o + g.pz) : 0.0;
        const double bz = zl ? at<PR>(g.b, o + g.pz) : 0.0;
        e += (a - az) * (b - bz);
      }
      // edges from the zero cells before index 0 of each dimension
      const int lower = (x == 0) + (y == 0) + (g.zdim && z == 0);
      e += lower * (a * b);
      acc += (a - b) * (a - b) + g.r2 * e;
    }
  }
  const double s = block_sum(acc, lds);
  if (threadIdx.x == 0) g.partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void energy_sum_kernel(const double *partial, int n,
                                                              double *out) {
  __shared__ double lds[kThreads / 64];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) v += partial[i];
  const double s = block_sum(v, lds);
  if (threadIdx.x == 0) *out = s;
}

template <class PR>
void launch(const EnergyArgs &g, int blocks, double *out, hipStream_t s) {
  hipLaunchKernelGGL(energy_kernel<PR>, dim3(blocks), dim3(kThreads), 0, s, g);
  hipLaunchKernelGGL(energy_sum_kernel, dim3(1), dim3(kThreads), 0, s, g.partial, blocks, out);
}

}  // namespace
}  // namespace ccl

using namespace ccl;

extern "C" ccl_status ccl_wave_energy(int32_t dims, const int64_t *shape, const int64_t *pitch,
                                      int32_t dtype, double r2, const void *u_new,
                                      const void *u_old, double *energy_out, void *hip_stream) {
  clear_error();
  if (dims != 2 && dims != 3) return fail(CCL_E_INVALID, "dims=%d (2 or 3)", dims);
  if (!shape || !pitch || !u_new || !u_old || !energy_out)
    return fail(CCL_E_INVALID, "NULL argument");
  if (dtype_bytes(dtype) == 0) return fail(CCL_E_INVALID, "unknown dtype %d", dtype);
  for (int d = 0; d < dims; ++d)
    if (shape[d] < 1) return fail(CCL_E_INVALID, "shape[%d]=%lld < 1", d, (long long)shape[d]);
  EnergyArgs g;
  g.a = u_new;
  g.b = u_old;
  g.zdim = dims == 3;
  g.nz = dims == 3 ? shape[0] : 1;
  g.ny = shape[dims - 2];
  g.nx = shape[dims - 1];
  g.py = pitch[dims - 2];
  g.pz = dims == 3 ? pitch[0] : g.py * g.ny;
  if (g.py < g.nx || (dims == 3 && g.pz < g.py * g.ny))
    return fail(CCL_E_INVALID, "pitches smaller than the rows or planes they hold");
  g.r2 = r2;
  const int64_t rows = g.nz * g.ny;
  const int blocks = static_cast<int>(std::min<int64_t>(rows, kMaxBlocks));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  double *partial = nullptr;
  ccl_status st = hip_check(hipMallocAsync(reinterpret_cast<void **>(&partial),
                                           sizeof(double) * blocks, s),
                            "hipMallocAsync(energy partials)");
  if (st != CCL_OK) return st;
  g.partial = partial;
  switch (dtype) {
    case CCL_DTYPE_F64: launch<P64>(g, blocks, energy_out, s); break;
    case CCL_DTYPE_BF16: launch<PB16>(g, blocks, energy_out, s); break;
    case CCL_DTYPE_F16: launch<PH16>(g, blocks, energy_out, s); break;
    default: launch<P32>(g, blocks, energy_out, s); break;
  }
  st = hip_check(hipGetLastError(), "energy_kernel launch");
  const ccl_status fs = hip_check(hipFreeAsync(partial, s), "hipFreeAsync(energy partials)");
  return st != CCL_OK ? st : fs;
}
