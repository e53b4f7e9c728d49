// Device-local transfers between chunk buffers (section 3: the regions a
// chunk needs but does not own are copied in before it runs), plus packing
// of such boxes into a contiguous staging buffer and back.
//
// Every copy is a list of jobs; a job is a 3-level box of units (n0 x n1
// rows of n2 contiguous units; a unit is 4 bytes, or 2 for 2-byte
// elements).  One launch serves up to kJobsPerLaunch jobs: the rows of all
// jobs are cut into segments of at most kSegUnits units and each wave copies
// one segment at a time, with 16-byte accesses when both row addresses
// allow it.
#include <cstring>
#include <vector>

#include "ccl_internal.h"

namespace ccl {
namespace {

constexpr int kJobsPerLaunch = 32;
constexpr int kSegUnits = 512;
constexpr int kThreads = 256;

struct CopyArgs {
  int32_t njobs;
  int64_t task_begin[kJobsPerLaunch + 1];
  CopyJob jobs[kJobsPerLaunch];
};

// One row segment of `len` units of type U (16-byte words where both ends
// are aligned and the length allows it).
template <class U>
__device__ __forceinline__ void copy_row(const U *src, U *dst, int64_t len, int lane) {
  constexpr int per16 = 16 / sizeof(U);
  const bool vec = ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15u) == 0 &&
                   (len % per16) == 0;
  if (vec) {
    const uint4 *s4 = reinterpret_cast<const uint4 *>(src);
    uint4 *d4 = reinterpret_cast<uint4 *>(dst);
    const int64_t n4 = len / per16;
    for (int64_t q = lane; q < n4; q += 64) d4[q] = s4[q];
  } else {
    for (int64_t q = lane; q < len; q += 64) dst[q] = src[q];
  }
}

__global__ __launch_bounds__(kThreads) void copy_boxes_kernel(CopyArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t wave0 = (static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * kThreads) >> 6;
  const int64_t ntasks = a.task_begin[a.njobs];
  for (int64_t t = __builtin_amdgcn_readfirstlane(static_cast<int>(wave0)); t < ntasks;
       t += nwaves) {
    int j = 0;
    while (j + 1 < a.njobs && t >= a.task_begin[j + 1]) ++j;
    const CopyJob &J = a.jobs[j];
    const int64_t local = t - a.task_begin[j];
    const int64_t segs = (J.n2 + kSegUnits - 1) / kSegUnits;
    const int64_t row = local / segs;
    const int64_t seg = local - row * segs;
    const int64_t i0 = row / J.n1;
    const int64_t i1 = row - i0 * J.n1;
    const int64_t w0 = seg * kSegUnits;
    const int64_t len = (J.n2 - w0) < kSegUnits ? (J.n2 - w0) : kSegUnits;
    const int64_t so = i0 * J.src_pitch0 + i1 * J.src_pitch1 + w0;
    const int64_t dof = i0 * J.dst_pitch0 + i1 * J.dst_pitch1 + w0;
    if (J.unit == 4)
      copy_row(static_cast<const uint32_t *>(J.src) + so, static_cast<uint32_t *>(J.dst) + dof,
               len, lane);
    else
      copy_row(static_cast<const uint16_t *>(J.src) + so, static_cast<uint16_t *>(J.dst) + dof,
               len, lane);
  }
}

}  // namespace

ccl_status launch_copies(const CopyJob *jobs, int32_t njobs, hipStream_t stream) {
  int32_t done = 0;
  while (done < njobs) {
    CopyArgs a;
    memset(&a, 0, sizeof(a));
    int64_t tasks = 0;
    a.task_begin[0] = 0;
    for (; done < njobs && a.njobs < kJobsPerLaunch; ++done) {
      const CopyJob &J = jobs[done];
      if (J.n0 <= 0 || J.n1 <= 0 || J.n2 <= 0) continue;
      a.jobs[a.njobs] = J;
      tasks += static_cast<int64_t>(J.n0) * J.n1 * ((J.n2 + kSegUnits - 1) / kSegUnits);
      a.task_begin[++a.njobs] = tasks;
    }
    if (a.njobs == 0) continue;
    const int64_t waves_per_block = kThreads / 64;
    int64_t blocks = (tasks + waves_per_block - 1) / waves_per_block;
    if (blocks > 4096) blocks = 4096;
    if (tasks > (int64_t(1) << 31)) return fail(CCL_E_RANGE, "copy too large for one launch");
    {
      TimedLaunch tl(CCL_KERNEL_HALO, stream);
      hipLaunchKernelGGL(copy_boxes_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kThreads),
                         0, stream, a);
    }
    ccl_status st = hip_check(hipGetLastError(), "copy_boxes_kernel launch");
    if (st != CCL_OK) return st;
  }
  return CCL_OK;
}

// Units of a box copy for elements of `elem_bytes` bytes: 4 bytes when
// the element size allows, else 2.
static int32_t unit_of(int32_t elem_bytes) { return (elem_bytes % 4) == 0 ? 4 : 2; }

// Builds the job that copies `box` (global indices) from src to dst buffers,
// upe units per element of `unit` bytes.
static ccl_status box_job(const Box &box, const void *src_base, const Box &src_reg,
                          const int64_t *src_pitch, void *dst_base, const Box &dst_reg,
                          const int64_t *dst_pitch, int32_t unit, int32_t upe, CopyJob *job) {
  const int dims = box.dims;
  int64_t soff = 0, doff = 0;
  for (int d = 0; d < dims; ++d) {
    soff += (box.lo[d] - src_reg.lo[d]) * src_pitch[d];
    doff += (box.lo[d] - dst_reg.lo[d]) * dst_pitch[d];
  }
  CopyJob J;
  J.unit = unit;
  J.src = static_cast<const char *>(src_base) + soff * upe * unit;
  J.dst = static_cast<char *>(dst_base) + doff * upe * unit;
  int64_t ext[3] = {1, 1, 1}, sp[3] = {0, 0, 0}, dp[3] = {0, 0, 0};
  // right-align the box into a 3-level (n0, n1, n2) shape
  for (int d = 0; d < dims; ++d) {
    const int k = 3 - dims + d;
    ext[k] = box.hi[d] - box.lo[d];
    sp[k] = src_pitch[d] * upe;
    dp[k] = dst_pitch[d] * upe;
  }
  ext[2] *= upe;
  if (ext[0] > INT32_MAX || ext[1] > INT32_MAX || ext[2] > INT32_MAX)
    return fail(CCL_E_RANGE, "box too large");
  J.n0 = static_cast<int32_t>(ext[0]);
  J.n1 = static_cast<int32_t>(ext[1]);
  J.n2 = static_cast<int32_t>(ext[2]);
  J.src_pitch0 = sp[0];
  J.src_pitch1 = sp[1];
  J.dst_pitch0 = dp[0];
  J.dst_pitch1 = dp[1];
  *job = J;
  return CCL_OK;
}

static ccl_status pack_like(int32_t nboxes, const ccl_subrange *boxes,
                            const ccl_chunk_buffer *bufs, int32_t elem_bytes, void *staging,
                            bool pack, void *hip_stream) {
  clear_error();
  if (nboxes < 0 || (nboxes > 0 && (!boxes || !bufs || !staging)))
    return fail(CCL_E_INVALID, "NULL argument or negative count");
  if (elem_bytes <= 0 || (elem_bytes % 2) != 0)
    return fail(CCL_E_INVALID, "elem_bytes=%d must be a positive multiple of 2", elem_bytes);
  const int32_t unit = unit_of(elem_bytes), upe = elem_bytes / unit;
  if ((reinterpret_cast<uintptr_t>(staging) & static_cast<uintptr_t>(unit - 1)) != 0)
    return fail(CCL_E_INVALID, "staging must be %d-byte aligned", unit);
  std::vector<CopyJob> jobs;
  int64_t cursor = 0;  // in elements
  for (int b = 0; b < nboxes; ++b) {
    const ccl_chunk_buffer &B = bufs[b];
    const int dims = boxes[b].dims;
    if (dims < 1 || dims > CCL_MAX_DIMS) return fail(CCL_E_INVALID, "box %d dims=%d", b, dims);
    ccl_status st = check_buffer(B, dims, pack ? "pack source" : "unpack target", false);
    if (st != CCL_OK) return st;
    if ((reinterpret_cast<uintptr_t>(B.base) & static_cast<uintptr_t>(unit - 1)) != 0)
      return fail(CCL_E_INVALID, "buffer %d not %d-byte aligned", b, unit);
    Box box = box_of(boxes[b]);
    Box reg = box_of(B.region);
    if (!contains(reg, box)) return fail(CCL_E_RANGE, "box %d outside its buffer's region", b);
    int64_t vol = box.volume();
    if (vol == 0) continue;
    // staging side: the box packed densely, row-major
    int64_t spitch[CCL_MAX_DIMS];
    spitch[dims - 1] = 1;
    for (int d = dims - 2; d >= 0; --d) spitch[d] = spitch[d + 1] * (box.hi[d + 1] - box.lo[d + 1]);
    char *stg = static_cast<char *>(staging) + cursor * elem_bytes;
    CopyJob J;
    if (pack)
      st = box_job(box, B.base, reg, B.pitch, stg, box, spitch, unit, upe, &J);
    else
      st = box_job(box, stg, box, spitch, B.base, reg, B.pitch, unit, upe, &J);
    if (st != CCL_OK) return st;
    jobs.push_back(J);
    cursor += vol;
  }
  if (jobs.empty()) return CCL_OK;
  return launch_copies(jobs.data(), static_cast<int32_t>(jobs.size()),
                       static_cast<hipStream_t>(hip_stream));
}

// Jobs for every inferred transfer of `mapper` among the chunk buffers.
ccl_status exchange_jobs(int32_t nchunks, const ccl_chunk *chunks, const ccl_range_mapper &mapper,
                         const ccl_chunk_buffer *bufs, int32_t elem_bytes,
                         std::vector<CopyJob> *jobs) {
  const int dims = chunks[0].dims;
  const int32_t unit = unit_of(elem_bytes), upe = elem_bytes / unit;
  // buffer range: the chunks' regions are clipped to the domain, which
  // already lies inside the buffer; clipping to the domain gives the same
  // boxes because a transfer box always lies inside the owner chunk.
  // (the chunks' global range starts at or above 0 and ends at `upto`)
  int64_t upto[CCL_MAX_DIMS] = {1, 1, 1};
  const Box dom = domain_box(chunks[0]);
  for (int d = 0; d < dims; ++d) upto[d] = dom.hi[d];
  for (int j = 0; j < nchunks; ++j) {
    Box need;
    ccl_status st = region_box(chunks[j], mapper, upto, &need);
    if (st != CCL_OK) return st;
    for (int k = 0; k < nchunks; ++k) {
      if (k == j) continue;
      Box b = intersect(need, chunk_box(chunks[k]));
      if (b.empty()) continue;
      const Box rk = box_of(bufs[k].region), rj = box_of(bufs[j].region);
      if (!contains(rk, b))
        return fail(CCL_E_RANGE, "owner buffer %d does not hold the box it must send", k);
      if (!contains(rj, b))
        return fail(CCL_E_RANGE, "reader buffer %d region lacks the halo its mapper needs", j);
      CopyJob J;
      ccl_status st = box_job(b, bufs[k].base, rk, bufs[k].pitch, bufs[j].base, rj,
                              bufs[j].pitch, unit, upe, &J);
      if (st != CCL_OK) return st;
      jobs->push_back(J);
    }
  }
  return CCL_OK;
}

}  // namespace ccl

using namespace ccl;

extern "C" {

ccl_status ccl_halo_exchange(int32_t nchunks, const ccl_chunk *chunks,
                             const ccl_range_mapper *mapper, const ccl_chunk_buffer *bufs,
                             int32_t elem_bytes, void *hip_stream) {
  clear_error();
  if (!mapper || !bufs) return fail(CCL_E_INVALID, "NULL argument");
  if (elem_bytes <= 0 || (elem_bytes % 2) != 0)
    return fail(CCL_E_INVALID, "elem_bytes=%d must be a positive multiple of 2", elem_bytes);
  ccl_status st = check_chunks(nchunks, chunks, 0);
  if (st != CCL_OK) return st;
  const int dims = chunks[0].dims;
  const uintptr_t amask = (elem_bytes % 4) == 0 ? 3u : 1u;
  for (int k = 0; k < nchunks; ++k) {
    st = check_buffer(bufs[k], dims, "halo buffer", false);
    if (st != CCL_OK) return st;
    if ((reinterpret_cast<uintptr_t>(bufs[k].base) & amask) != 0)
      return fail(CCL_E_INVALID, "buffer %d not %d-byte aligned", k, static_cast<int>(amask + 1));
    if (!contains(box_of(bufs[k].region), chunk_box(chunks[k])))
      return fail(CCL_E_RANGE, "buffer %d does not hold its chunk", k);
  }
  std::vector<CopyJob> jobs;
  st = exchange_jobs(nchunks, chunks, *mapper, bufs, elem_bytes, &jobs);
  if (st != CCL_OK) return st;
  if (jobs.empty()) return CCL_OK;
  return launch_copies(jobs.data(), static_cast<int32_t>(jobs.size()),
                       static_cast<hipStream_t>(hip_stream));
}

ccl_status ccl_halo_pack(int32_t nboxes, const ccl_subrange *boxes, const ccl_chunk_buffer *srcs,
                         int32_t elem_bytes, void *staging, void *hip_stream) {
  return pack_like(nboxes, boxes, srcs, elem_bytes, staging, true, hip_stream);
}

ccl_status ccl_halo_unpack(int32_t nboxes, const ccl_subrange *boxes,
                           const ccl_chunk_buffer *dsts, int32_t elem_bytes,
                           const void *staging, void *hip_stream) {
  return pack_like(nboxes, boxes, dsts, elem_bytes, const_cast<void *>(staging), false,
                   hip_stream);
}

}  // extern "C"
