// Range splitting, range mappers and transfer inference (host side).
//
// Section 3 of the paper: a kernel's execution range is split into chunks,
// one per device, and each accessor's range mapper maps a chunk to the
// region of the buffer it touches; the parts of those regions that another
// chunk owns are the transfers the runtime performs before the kernel runs.
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "ccl_internal.h"

namespace ccl {

static thread_local char g_err[512] = {0};

ccl_status fail(ccl_status st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

void clear_error() { g_err[0] = 0; }

Box box_of(const ccl_subrange &s) {
  Box b;
  b.dims = s.dims;
  for (int d = 0; d < s.dims && d < CCL_MAX_DIMS; ++d) {
    b.lo[d] = s.offset[d];
    b.hi[d] = s.offset[d] + s.range[d];
  }
  return b;
}

Box chunk_box(const ccl_chunk &c) {
  Box b;
  b.dims = c.dims;
  for (int d = 0; d < c.dims; ++d) {
    b.lo[d] = c.offset[d];
    b.hi[d] = c.offset[d] + c.range[d];
  }
  return b;
}

Box domain_box(const ccl_chunk &c) {
  Box b;
  b.dims = c.dims;
  for (int d = 0; d < c.dims; ++d) {
    b.lo[d] = c.global_offset[d];
    b.hi[d] = c.global_offset[d] + c.global_range[d];
  }
  return b;
}

ccl_subrange subrange_of(const Box &b) {
  ccl_subrange s;
  memset(&s, 0, sizeof(s));
  s.dims = b.dims;
  for (int d = 0; d < b.dims; ++d) {
    s.offset[d] = b.lo[d];
    s.range[d] = b.hi[d] > b.lo[d] ? b.hi[d] - b.lo[d] : 0;
  }
  return s;
}

Box intersect(const Box &a, const Box &b) {
  Box r;
  r.dims = a.dims;
  for (int d = 0; d < a.dims; ++d) {
    r.lo[d] = a.lo[d] > b.lo[d] ? a.lo[d] : b.lo[d];
    r.hi[d] = a.hi[d] < b.hi[d] ? a.hi[d] : b.hi[d];
    if (r.hi[d] < r.lo[d]) r.hi[d] = r.lo[d];
  }
  return r;
}

bool contains(const Box &outer, const Box &inner) {
  if (inner.empty()) return true;
  for (int d = 0; d < inner.dims; ++d)
    if (inner.lo[d] < outer.lo[d] || inner.hi[d] > outer.hi[d]) return false;
  return true;
}

Box grow(const Box &b, int64_t e) {
  Box r = b;
  for (int d = 0; d < b.dims; ++d) {
    r.lo[d] -= e;
    r.hi[d] += e;
  }
  return r;
}

ccl_status check_chunks(int32_t nchunks, const ccl_chunk *chunks, int32_t dims) {
  if (!chunks) return fail(CCL_E_INVALID, "chunks is NULL");
  if (nchunks < 1 || nchunks > CCL_MAX_CHUNKS)
    return fail(CCL_E_INVALID, "nchunks=%d outside [1,%d]", nchunks, CCL_MAX_CHUNKS);
  for (int k = 0; k < nchunks; ++k) {
    const ccl_chunk &c = chunks[k];
    if (c.dims != dims && dims > 0)
      return fail(CCL_E_INVALID, "chunk %d has dims=%d, expected %d", k, c.dims, dims);
    if (c.dims < 1 || c.dims > CCL_MAX_DIMS)
      return fail(CCL_E_INVALID, "chunk %d has dims=%d", k, c.dims);
    for (int d = 0; d < c.dims; ++d) {
      if (c.range[d] < 1 || c.global_range[d] < 1)
        return fail(CCL_E_INVALID, "chunk %d has an empty extent in dim %d", k, d);
    }
    if (!contains(domain_box(c), chunk_box(c)))
      return fail(CCL_E_RANGE, "chunk %d is not inside its global range", k);
    for (int d = 0; d < c.dims; ++d)
      if (c.global_offset[d] != chunks[0].global_offset[d] ||
          c.global_range[d] != chunks[0].global_range[d])
        return fail(CCL_E_INVALID, "chunks %d and 0 come from different ranges", k);
  }
  for (int a = 0; a < nchunks; ++a)
    for (int b = a + 1; b < nchunks; ++b)
      if (!intersect(chunk_box(chunks[a]), chunk_box(chunks[b])).empty())
        return fail(CCL_E_RANGE, "chunks %d and %d overlap", a, b);
  return CCL_OK;
}

ccl_status check_buffer(const ccl_chunk_buffer &b, int32_t dims, const char *what,
                        bool need_vec_align) {
  if (!b.base) return fail(CCL_E_INVALID, "%s: base is NULL", what);
  if (b.region.dims != dims)
    return fail(CCL_E_INVALID, "%s: region dims=%d, expected %d", what, b.region.dims, dims);
  for (int d = 0; d < dims; ++d)
    if (b.region.range[d] < 1)
      return fail(CCL_E_INVALID, "%s: empty region in dim %d", what, d);
  if (b.pitch[dims - 1] != 1)
    return fail(CCL_E_INVALID, "%s: innermost pitch must be 1", what);
  for (int d = 0; d + 1 < dims; ++d) {
    // each step of dim d must clear the whole extent of dim d+1
    if (b.pitch[d] < b.region.range[d + 1] * b.pitch[d + 1])
      return fail(CCL_E_INVALID, "%s: pitch[%d]=%lld too small", what, d, (long long)b.pitch[d]);
    if (need_vec_align && (b.pitch[d] % 4) != 0)
      return fail(CCL_E_INVALID, "%s: pitch[%d] must be a multiple of 4 elements", what, d);
  }
  if (need_vec_align && (reinterpret_cast<uintptr_t>(b.base) & 15u) != 0)
    return fail(CCL_E_INVALID, "%s: base must be 16-byte aligned", what);
  return CCL_OK;
}

ccl_status region_box(const ccl_chunk &c, const ccl_range_mapper &m, const int64_t *buffer_range,
                      Box *out) {
  Box r;
  r.dims = c.dims;
  switch (m.kind) {
    case CCL_MAP_ONE_TO_ONE:
      r = chunk_box(c);
      break;
    case CCL_MAP_NEIGHBORHOOD:
      for (int d = 0; d < c.dims; ++d) {
        if (m.extent[d] < 0) return fail(CCL_E_INVALID, "negative neighborhood extent");
        int64_t lo = c.offset[d] - m.extent[d];
        int64_t hi = c.offset[d] + c.range[d] + m.extent[d];
        r.lo[d] = lo < 0 ? 0 : lo;
        r.hi[d] = hi > buffer_range[d] ? buffer_range[d] : hi;
        if (r.hi[d] < r.lo[d]) r.hi[d] = r.lo[d];
      }
      break;
    case CCL_MAP_ALL:
      for (int d = 0; d < c.dims; ++d) {
        r.lo[d] = 0;
        r.hi[d] = buffer_range[d];
      }
      break;
    case CCL_MAP_FIXED:
      for (int d = 0; d < c.dims; ++d) {
        if (m.extent[d] < 0) return fail(CCL_E_INVALID, "negative fixed extent");
        const int64_t lo = m.offset[d], hi = m.offset[d] + m.extent[d];
        r.lo[d] = lo < 0 ? 0 : lo > buffer_range[d] ? buffer_range[d] : lo;
        r.hi[d] = hi > buffer_range[d] ? buffer_range[d] : hi < r.lo[d] ? r.lo[d] : hi;
      }
      break;
    case CCL_MAP_SLICE:
      if (m.dim < 0 || m.dim >= c.dims)
        return fail(CCL_E_INVALID, "slice dim=%d not in [0,%d)", m.dim, c.dims);
      r = chunk_box(c);
      r.lo[m.dim] = 0;
      r.hi[m.dim] = buffer_range[m.dim];
      break;
    default:
      return fail(CCL_E_INVALID, "unknown range mapper kind %d", m.kind);
  }
  *out = r;
  return CCL_OK;
}

}  // namespace ccl

using namespace ccl;

extern "C" {

const char *ccl_version(void) { return "libccl 0.1 (gfx950)"; }

const char *ccl_last_error(void) { return g_err; }

ccl_status ccl_split_range(const ccl_subrange *range, int32_t nchunks, int32_t split_dim,
                           ccl_chunk *chunks_out) {
  clear_error();
  if (!range || !chunks_out) return fail(CCL_E_INVALID, "NULL argument");
  const int dims = range->dims;
  if (dims < 1 || dims > CCL_MAX_DIMS) return fail(CCL_E_INVALID, "dims=%d not in 1..3", dims);
  if (nchunks < 1) return fail(CCL_E_INVALID, "nchunks=%d < 1", nchunks);
  if (split_dim < 0 || split_dim >= dims)
    return fail(CCL_E_INVALID, "split_dim=%d not in [0,%d)", split_dim, dims);
  for (int d = 0; d < dims; ++d)
    if (range->range[d] < 1) return fail(CCL_E_INVALID, "empty range in dim %d", d);
  const int64_t n = range->range[split_dim];
  if (nchunks > n)
    return fail(CCL_E_RANGE, "nchunks=%d exceeds extent %lld of dim %d", nchunks,
                (long long)n, split_dim);
  for (int k = 0; k < nchunks; ++k) {
    ccl_chunk c;
    memset(&c, 0, sizeof(c));
    c.dims = dims;
    for (int d = 0; d < dims; ++d) {
      c.offset[d] = range->offset[d];
      c.range[d] = range->range[d];
      c.global_offset[d] = range->offset[d];
      c.global_range[d] = range->range[d];
    }
    const int64_t lo = (static_cast<int64_t>(k) * n) / nchunks;
    const int64_t hi = (static_cast<int64_t>(k + 1) * n) / nchunks;
    c.offset[split_dim] = range->offset[split_dim] + lo;
    c.range[split_dim] = hi - lo;
    chunks_out[k] = c;
  }
  return CCL_OK;
}

ccl_status ccl_split_grid(const ccl_subrange *range, const int32_t *counts,
                          ccl_chunk *chunks_out) {
  clear_error();
  if (!range || !counts || !chunks_out) return fail(CCL_E_INVALID, "NULL argument");
  const int dims = range->dims;
  if (dims < 1 || dims > CCL_MAX_DIMS) return fail(CCL_E_INVALID, "dims=%d not in 1..3", dims);
  int64_t total = 1;
  for (int d = 0; d < dims; ++d) {
    if (range->range[d] < 1) return fail(CCL_E_INVALID, "empty range in dim %d", d);
    if (counts[d] < 1) return fail(CCL_E_INVALID, "counts[%d]=%d < 1", d, counts[d]);
    if (counts[d] > range->range[d])
      return fail(CCL_E_RANGE, "counts[%d]=%d exceeds extent %lld", d, counts[d],
                  (long long)range->range[d]);
    total *= counts[d];
    if (total > (int64_t(1) << 30)) return fail(CCL_E_RANGE, "too many chunks");
  }
  for (int64_t k = 0; k < total; ++k) {
    ccl_chunk c;
    memset(&c, 0, sizeof(c));
    c.dims = dims;
    // chunk k's grid coordinates, last dimension fastest
    int64_t rest = k;
    for (int d = dims - 1; d >= 0; --d) {
      const int64_t kd = rest % counts[d];
      rest /= counts[d];
      const int64_t n = range->range[d];
      const int64_t lo = (kd * n) / counts[d];
      const int64_t hi = ((kd + 1) * n) / counts[d];
      c.offset[d] = range->offset[d] + lo;
      c.range[d] = hi - lo;
      c.global_offset[d] = range->offset[d];
      c.global_range[d] = range->range[d];
    }
    chunks_out[k] = c;
  }
  return CCL_OK;
}

ccl_status ccl_region_of(const ccl_chunk *chunk, const ccl_range_mapper *mapper,
                         const int64_t *buffer_range, ccl_subrange *region_out) {
  clear_error();
  if (!chunk || !mapper || !buffer_range || !region_out)
    return fail(CCL_E_INVALID, "NULL argument");
  if (chunk->dims < 1 || chunk->dims > CCL_MAX_DIMS)
    return fail(CCL_E_INVALID, "dims=%d not in 1..3", chunk->dims);
  for (int d = 0; d < chunk->dims; ++d)
    if (buffer_range[d] < 1) return fail(CCL_E_INVALID, "empty buffer range in dim %d", d);
  Box r;
  ccl_status st = region_box(*chunk, *mapper, buffer_range, &r);
  if (st != CCL_OK) return st;
  *region_out = subrange_of(r);
  return CCL_OK;
}

ccl_status ccl_transfers(int32_t nchunks, const ccl_chunk *chunks, const ccl_range_mapper *mapper,
                         const int64_t *buffer_range, ccl_transfer *out, int32_t capacity,
                         int32_t *count) {
  clear_error();
  if (!mapper || !buffer_range || !count) return fail(CCL_E_INVALID, "NULL argument");
  if (capacity < 0 || (capacity > 0 && !out)) return fail(CCL_E_INVALID, "bad capacity/out");
  ccl_status st = check_chunks(nchunks, chunks, 0);
  if (st != CCL_OK) return st;
  int32_t n = 0;
  for (int j = 0; j < nchunks; ++j) {
    Box reg;
    st = region_box(chunks[j], *mapper, buffer_range, &reg);
    if (st != CCL_OK) return st;
    for (int k = 0; k < nchunks; ++k) {
      if (k == j) continue;
      Box b = intersect(reg, chunk_box(chunks[k]));
      if (b.empty()) continue;
      if (n < capacity) {
        out[n].owner = k;
        out[n].reader = j;
        out[n].box = subrange_of(b);
      }
      ++n;
    }
  }
  *count = n;
  if (n > capacity) return fail(CCL_E_RANGE, "%d transfers exceed capacity %d", n, capacity);
  return CCL_OK;
}

}  // extern "C"
