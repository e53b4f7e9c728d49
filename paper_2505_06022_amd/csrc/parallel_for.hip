// Generic chunked parallel_for: one data-parallel function over an N-D
// range split into chunks, with accessors that carry a range mapper and an
// access mode (section 3, second listing and the paragraph after it).
//
// Before the function runs, every read accessor's inferred transfers are
// made: the part of region_of(chunk j, mapper) that chunk k owns is copied
// from chunk k's buffer into chunk j's (the same boxes ccl_halo_exchange
// copies).  Then one launch runs the function at every index of every
// chunk.  Each thread takes four consecutive indices along the innermost
// dimension; where every accessor's group of four is one aligned 16-byte
// word the thread moves it with one vector access, otherwise element by
// element.
#include <algorithm>
#include <cstring>
#include <vector>

#include "ccl_internal.h"

namespace ccl {
namespace {

constexpr int kMaxAcc = 3;
constexpr int kChunksPerLaunch = 8;
constexpr int kThreads = 256;

struct PFView {  // one accessor's buffer for one chunk
  float *base;
  int64_t off[CCL_MAX_DIMS];    // region origin (global indices)
  int64_t pitch[CCL_MAX_DIMS];  // element strides
};

struct PFChunk {
  int64_t lo[CCL_MAX_DIMS];  // chunk origin, unused dimensions 0
  int64_t n[CCL_MAX_DIMS];   // chunk extents, unused dimensions 1
  int64_t begin;             // first thread of this chunk in the launch
  int32_t vec;               // every accessor's quads are aligned 16-byte words
  PFView v[kMaxAcc];
};

struct PFArgs {
  int32_t nchunks;
  int32_t dims;
  int32_t sum_dim;  // CCL_FN_SUM_ALONG: the dimension summed
  float a;          // CCL_FN_SAXPY: the scalar
  int64_t total;    // threads in the launch
  int64_t sum_lo, sum_n;  // CCL_FN_SUM_ALONG: the range's extent along sum_dim
  PFChunk ch[kChunksPerLaunch];
};

__device__ __forceinline__ float *at(const PFView &v, int dims, const int64_t *i) {
  int64_t o = 0;
  for (int d = 0; d < dims; ++d) o += (i[d] - v.off[d]) * v.pitch[d];
  return v.base + o;
}

// z = fma(a, x, y) at one index (the function of the paper's first two
// listings); accessors: x (read), y (read), z (write).
__device__ __forceinline__ void saxpy_at(const PFChunk &C, int dims, float a, const int64_t *i) {
  *at(C.v[2], dims, i) = fmaf(a, *at(C.v[0], dims, i), *at(C.v[1], dims, i));
}

// out = x[.., 0, ..] + x[.., 1, ..] + ... along sum_dim, summed in index
// order from 0.0f; accessors: x (read, its region holds the whole extent
// along sum_dim: a SLICE or ALL mapper), out (write).
__device__ __forceinline__ void sum_at(const PFChunk &C, const PFArgs &a, const int64_t *i) {
  int64_t j[CCL_MAX_DIMS] = {i[0], i[1], i[2]};
  float acc = 0.0f;
  for (int64_t v = 0; v < a.sum_n; ++v) {
    j[a.sum_dim] = a.sum_lo + v;
    acc = acc + *at(C.v[0], a.dims, j);
  }
  *at(C.v[1], a.dims, i) = acc;
}

template <int FN>
__global__ __launch_bounds__(kThreads) void parallel_for_kernel(const PFArgs a) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (t >= a.total) return;
  int c = 0;
  while (c + 1 < a.nchunks && t >= a.ch[c + 1].begin) ++c;
  const PFChunk &C = a.ch[c];
  const int D = a.dims;
  // thread -> (outer indices, quad of four innermost indices)
  int64_t rest = t - C.begin;
  const int64_t nq = (C.n[D - 1] + 3) / 4;
  const int64_t q = rest % nq;
  rest /= nq;
  int64_t i[CCL_MAX_DIMS] = {0, 0, 0};
  for (int d = D - 2; d >= 0; --d) {
    i[d] = C.lo[d] + rest % C.n[d];
    rest /= C.n[d];
  }
  const int64_t x0 = C.lo[D - 1] + 4 * q;
  const int64_t x1 = min(x0 + 4, C.lo[D - 1] + C.n[D - 1]);
  if (FN == CCL_FN_SAXPY && C.vec && x1 - x0 == 4) {
    i[D - 1] = x0;
    const float4 x = *reinterpret_cast<const float4 *>(at(C.v[0], D, i));
    const float4 y = *reinterpret_cast<const float4 *>(at(C.v[1], D, i));
    float4 z;
    z.x = fmaf(a.a, x.x, y.x);
    z.y = fmaf(a.a, x.y, y.y);
    z.z = fmaf(a.a, x.z, y.z);
    z.w = fmaf(a.a, x.w, y.w);
    *reinterpret_cast<float4 *>(at(C.v[2], D, i)) = z;
    return;
  }
  for (int64_t x = x0; x < x1; ++x) {
    i[D - 1] = x;
    if (FN == CCL_FN_SAXPY)
      saxpy_at(C, D, a.a, i);
    else
      sum_at(C, a, i);
  }
}

bool is_read(int32_t m) { return m == CCL_ACCESS_READ || m == CCL_ACCESS_READ_WRITE; }
bool is_write(int32_t m) { return m == CCL_ACCESS_WRITE || m == CCL_ACCESS_READ_WRITE; }

}  // namespace
}  // namespace ccl

using namespace ccl;

extern "C" ccl_status ccl_parallel_for(const ccl_kernel_fn *fn, int32_t nchunks,
                                       const ccl_chunk *chunks, int32_t naccessors,
                                       const ccl_accessor *acc, void *hip_stream) {
  clear_error();
  if (!fn || !acc) return fail(CCL_E_INVALID, "NULL argument");
  ccl_status st = check_chunks(nchunks, chunks, 0);
  if (st != CCL_OK) return st;
  const int dims = chunks[0].dims;
  // the function's signature: accessor count and the mode each needs
  int want_n = 0;
  bool reads[kMaxAcc] = {false, false, false};
  switch (fn->fn) {
    case CCL_FN_SAXPY:
      want_n = 3;
      reads[0] = reads[1] = true;
      break;
    case CCL_FN_SUM_ALONG:
      want_n = 2;
      reads[0] = true;
      if (fn->dim < 0 || fn->dim >= dims)
        return fail(CCL_E_INVALID, "sum dimension %d not in [0,%d)", fn->dim, dims);
      break;
    default:
      return fail(CCL_E_INVALID, "unknown function %d", fn->fn);
  }
  if (naccessors != want_n)
    return fail(CCL_E_INVALID, "function %d takes %d accessors, got %d", fn->fn, want_n,
                naccessors);
  const Box dom = domain_box(chunks[0]);
  for (int b = 0; b < naccessors; ++b) {
    const ccl_accessor &A = acc[b];
    if (!A.bufs) return fail(CCL_E_INVALID, "accessor %d: NULL buffers", b);
    if (reads[b] && !is_read(A.mode))
      return fail(CCL_E_INVALID, "accessor %d must be readable", b);
    if (!reads[b]) {
      if (!is_write(A.mode)) return fail(CCL_E_INVALID, "accessor %d must be writable", b);
      if (A.mapper.kind != CCL_MAP_ONE_TO_ONE)
        return fail(CCL_E_INVALID, "accessor %d: the function writes only at its own index, "
                                   "so its mapper must be ONE_TO_ONE", b);
    }
    for (int d = 0; d < dims; ++d)
      if (A.buffer_range[d] < dom.hi[d])
        return fail(CCL_E_RANGE, "accessor %d: the kernel range is outside the buffer", b);
    for (int k = 0; k < nchunks; ++k) {
      st = check_buffer(A.bufs[k], dims, "accessor buffer", false);
      if (st != CCL_OK) return st;
      if ((reinterpret_cast<uintptr_t>(A.bufs[k].base) & 3u) != 0)
        return fail(CCL_E_INVALID, "accessor %d chunk %d: base not 4-byte aligned", b, k);
      Box need;
      st = region_box(chunks[k], A.mapper, A.buffer_range, &need);
      if (st != CCL_OK) return st;
      const Box reg = box_of(A.bufs[k].region);
      if (!contains(reg, need) || !contains(reg, chunk_box(chunks[k])))
        return fail(CCL_E_RANGE, "accessor %d chunk %d: buffer region lacks the mapper's region",
                    b, k);
      if (fn->fn == CCL_FN_SUM_ALONG && b == 0 &&
          (need.lo[fn->dim] > dom.lo[fn->dim] || need.hi[fn->dim] < dom.hi[fn->dim]))
        return fail(CCL_E_RANGE, "accessor 0 chunk %d: the mapper's region does not span the "
                                 "range along the summed dimension", k);
    }
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // 1. inferred transfers of the read accessors
  std::vector<CopyJob> jobs;
  for (int b = 0; b < naccessors; ++b) {
    if (!reads[b] || acc[b].mapper.kind == CCL_MAP_ONE_TO_ONE || nchunks == 1) continue;
    st = exchange_jobs(nchunks, chunks, acc[b].mapper, acc[b].bufs, 4, &jobs);
    if (st != CCL_OK) return st;
  }
  if (!jobs.empty()) {
    st = launch_copies(jobs.data(), static_cast<int32_t>(jobs.size()), s);
    if (st != CCL_OK) return st;
  }
  // 2. the function over every index of every chunk
  for (int first = 0; first < nchunks; first += kChunksPerLaunch) {
    const int n = std::min(kChunksPerLaunch, nchunks - first);
    PFArgs a;
    memset(&a, 0, sizeof(a));
    a.nchunks = n;
    a.dims = dims;
    a.a = fn->a;
    a.sum_dim = fn->fn == CCL_FN_SUM_ALONG ? fn->dim : 0;
    a.sum_lo = dom.lo[a.sum_dim];
    a.sum_n = dom.hi[a.sum_dim] - dom.lo[a.sum_dim];
    int64_t total = 0;
    for (int k = 0; k < n; ++k) {
      const ccl_chunk &c = chunks[first + k];
      PFChunk &C = a.ch[k];
      for (int d = 0; d < CCL_MAX_DIMS; ++d) {
        C.lo[d] = d < dims ? c.offset[d] : 0;
        C.n[d] = d < dims ? c.range[d] : 1;
      }
      C.begin = total;
      int64_t threads = (C.n[dims - 1] + 3) / 4;
      for (int d = 0; d + 1 < dims; ++d) threads *= C.n[d];
      total += threads;
      C.vec = 1;
      for (int b = 0; b < naccessors; ++b) {
        const ccl_chunk_buffer &B = acc[b].bufs[first + k];
        PFView &V = C.v[b];
        V.base = static_cast<float *>(B.base);
        for (int d = 0; d < CCL_MAX_DIMS; ++d) {
          V.off[d] = d < dims ? B.region.offset[d] : 0;
          V.pitch[d] = d < dims ? B.pitch[d] : 0;
        }
        // quads start at the chunk's first column: vector accesses need it,
        // the base and every outer stride on 16-byte boundaries
        bool ok = (reinterpret_cast<uintptr_t>(B.base) & 15u) == 0 &&
                  ((c.offset[dims - 1] - B.region.offset[dims - 1]) % 4) == 0;
        for (int d = 0; d + 1 < dims; ++d) ok = ok && (B.pitch[d] % 4) == 0;
        if (!ok) C.vec = 0;
      }
    }
    a.total = total;
    if (total == 0) continue;
    const int64_t blocks = (total + kThreads - 1) / kThreads;
    if (blocks > INT32_MAX) return fail(CCL_E_RANGE, "range too large for one launch");
    if (fn->fn == CCL_FN_SAXPY) {
      TimedLaunch tl(CCL_KERNEL_SAXPY, s);
      hipLaunchKernelGGL(parallel_for_kernel<CCL_FN_SAXPY>, dim3(static_cast<unsigned>(blocks)),
                         dim3(kThreads), 0, s, a);
    } else {
      hipLaunchKernelGGL(parallel_for_kernel<CCL_FN_SUM_ALONG>,
                         dim3(static_cast<unsigned>(blocks)), dim3(kThreads), 0, s, a);
    }
    st = hip_check(hipGetLastError(), "parallel_for_kernel launch");
    if (st != CCL_OK) return st;
  }
  return CCL_OK;
}
