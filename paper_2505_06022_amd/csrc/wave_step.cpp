// ccl_wave_step: blocks of T leapfrog steps over device-local chunks.
//
// Before each block the halos the range mappers call for are copied in
// (NEIGHBORHOOD(T) of u^n, NEIGHBORHOOD(T-1) of u^{n-1}: section 3, the
// transfers inferred from the mappers), then one launch advances every chunk
// T steps.  The host only plans and enqueues; the caller's descriptor arrays
// are rotated to name the newest levels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <utility>
#include <vector>

#include "ccl_internal.h"

namespace ccl {

namespace {

WaveField field_of(const ccl_chunk_buffer &b) {
  WaveField f;
  f.base = b.base;
  for (int d = 0; d < CCL_MAX_DIMS; ++d) {
    f.off[d] = d < b.region.dims ? b.region.offset[d] : 0;
    f.pitch[d] = d < b.region.dims ? b.pitch[d] : 0;
  }
  return f;
}

// Region requirement of a role: chunk grown by `e`, clipped to the domain.
bool holds(const ccl_chunk_buffer &b, const ccl_chunk &c, int64_t e) {
  Box need = intersect(grow(chunk_box(c), e), domain_box(c));
  return contains(box_of(b.region), need);
}

// Every chunk spans the domain's full width: a split along rows (2D).
bool row_split(int32_t nchunks, const ccl_chunk *chunks) {
  for (int k = 0; k < nchunks; ++k) {
    const Box c = chunk_box(chunks[k]), d = domain_box(chunks[k]);
    if (c.lo[1] != d.lo[1] || c.hi[1] != d.hi[1]) return false;
  }
  return true;
}

// The halo rows chunk k's launch can store straight into the other chunks'
// output buffers for the next block of `next` steps: the rows of chunk k
// within `next` (u^{n+T}) and `next` - 1 (u^{n+T-1}) rows of chunk j, the
// boxes the exchange before that block would copy.  False (no pushes) if a
// chunk has more neighbours than a plan holds.
bool plan_pushes(int32_t nchunks, const ccl_chunk *chunks, const ccl_chunk_buffer *out_cur,
                 const ccl_chunk_buffer *out_prev, int next, WaveChunkPlan *plans) {
  for (int k = 0; k < nchunks; ++k) plans[k].npush = 0;
  for (int k = 0; k < nchunks; ++k) {
    const Box ck = chunk_box(chunks[k]);
    for (int j = 0; j < nchunks; ++j) {
      if (j == k) continue;
      const Box cj = chunk_box(chunks[j]);
      PushPlan Q;
      Q.cr0 = std::max(ck.lo[0], cj.lo[0] - next);
      Q.cr1 = std::min(ck.hi[0], cj.hi[0] + next);
      Q.pr0 = std::max(ck.lo[0], cj.lo[0] - (next - 1));
      Q.pr1 = std::min(ck.hi[0], cj.hi[0] + (next - 1));
      if (!out_prev) Q.pr1 = Q.pr0;  // in place: u^{n-1} of the next block needs no halo
      if (Q.cr1 <= Q.cr0 && Q.pr1 <= Q.pr0) continue;
      if (plans[k].npush == kMaxPushPerChunk) return false;
      Q.cur = field_of(out_cur[j]);
      Q.prev = out_prev ? field_of(out_prev[j]) : Q.cur;
      plans[k].push[plans[k].npush++] = Q;
    }
  }
  return true;
}

}  // namespace
}  // namespace ccl

using namespace ccl;

extern "C" ccl_status ccl_wave_step(const ccl_wave_params *p, int32_t nchunks,
                                    const ccl_chunk *chunks, ccl_chunk_buffer *u_prev,
                                    ccl_chunk_buffer *u_cur, ccl_chunk_buffer *w_prev,
                                    ccl_chunk_buffer *w_cur, int32_t nsteps, void *hip_stream) {
  clear_error();
  if (!p || !u_prev || !u_cur) return fail(CCL_E_INVALID, "NULL argument");
  const int dims = p->dims;
  if (dims != 2 && dims != 3) return fail(CCL_E_INVALID, "wave dims=%d must be 2 or 3", dims);
  if (!std::isfinite(p->r2) || p->r2 < 0.0) return fail(CCL_E_INVALID, "r2 must be finite, >= 0");
  const int32_t dtype = p->dtype;
  const int esize = dtype_bytes(dtype);
  if (esize == 0) return fail(CCL_E_INVALID, "dtype=%d unknown", dtype);
  if (dtype != CCL_DTYPE_F64 && !std::isfinite(static_cast<float>(p->r2)))
    return fail(CCL_E_INVALID, "r2 overflows float");
  const int T = p->temporal_depth;
  if (T < 1 || T > CCL_MAX_DEPTH)
    return fail(CCL_E_INVALID, "temporal_depth=%d not in 1..%d", T, CCL_MAX_DEPTH);
  if (p->tile_rows < 0) return fail(CCL_E_INVALID, "tile_rows < 0");
  if (p->flags != 0) return fail(CCL_E_INVALID, "flags must be 0");
  if (nsteps < 0) return fail(CCL_E_INVALID, "nsteps < 0");
  ccl_status st = check_chunks(nchunks, chunks, dims);
  if (st != CCL_OK) return st;
  const bool need_w = T > 1 && nsteps > 1;
  if (need_w && (!w_prev || !w_cur))
    return fail(CCL_E_INVALID, "T > 1 needs the w_prev / w_cur buffer pair");
  for (int k = 0; k < nchunks; ++k) {
    ccl_chunk_buffer *sets[4] = {u_prev, u_cur, need_w ? w_prev : nullptr,
                                 need_w ? w_cur : nullptr};
    const char *names[4] = {"u_prev", "u_cur", "w_prev", "w_cur"};
    // each lane group (dtype_group elements) must be one aligned access
    const int group = dtype_group(dtype);
    const uintptr_t amask = static_cast<uintptr_t>(group * esize - 1);
    for (int b = 0; b < 4; ++b) {
      if (!sets[b]) continue;
      st = check_buffer(sets[b][k], dims, names[b], false);
      if (st != CCL_OK) return st;
      for (int d = 0; d + 1 < dims; ++d)
        if (sets[b][k].pitch[d] % group != 0)
          return fail(CCL_E_INVALID, "%s: pitch[%d] must be a multiple of %d elements", names[b],
                      d, group);
      if ((reinterpret_cast<uintptr_t>(sets[b][k].base) & amask) != 0)
        return fail(CCL_E_INVALID, "%s: base must be %d-byte aligned", names[b],
                    static_cast<int>(amask + 1));
    }
  }
  if (nsteps == 0) return CCL_OK;

  // Dry run of the role rotation: check every block's region requirements
  // before anything is enqueued.
  {
    std::vector<ccl_chunk_buffer> up(u_prev, u_prev + nchunks), uc(u_cur, u_cur + nchunks);
    std::vector<ccl_chunk_buffer> wp, wc;
    if (need_w) {
      wp.assign(w_prev, w_prev + nchunks);
      wc.assign(w_cur, w_cur + nchunks);
    }
    for (int done = 0; done < nsteps;) {
      const int tb = (nsteps - done) < T ? (nsteps - done) : T;
      for (int k = 0; k < nchunks; ++k) {
        if (!holds(uc[k], chunks[k], tb))
          return fail(CCL_E_RANGE, "chunk %d: u^n buffer region lacks the %d-wide halo", k, tb);
        if (!holds(up[k], chunks[k], tb - 1))
          return fail(CCL_E_RANGE, "chunk %d: u^{n-1} buffer region lacks the %d-wide halo", k,
                      tb - 1);
        if (tb > 1 && (!contains(box_of(wp[k].region), chunk_box(chunks[k])) ||
                       !contains(box_of(wc[k].region), chunk_box(chunks[k]))))
          return fail(CCL_E_RANGE, "chunk %d: w buffers do not hold the chunk", k);
      }
      if (tb == 1) {
        std::swap(up, uc);
      } else {
        std::swap(up, wp);
        std::swap(uc, wc);
      }
      done += tb;
    }
  }

  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  std::vector<WaveChunkPlan> plans(nchunks);
  std::vector<CopyJob> jobs;
  // 2D splits along rows: each launch also stores the rows the next block's
  // halos need into the neighbours' output buffers, so only the first block
  // runs the exchange (the same boxes, the same values)
  const bool can_push = dims == 2 && nchunks > 1 && row_split(nchunks, chunks);
  bool halos_ready = false;
  for (int done = 0; done < nsteps;) {
    const int tb = (nsteps - done) < T ? (nsteps - done) : T;
    const bool in_place = tb == 1;
    const int next = std::min(T, nsteps - done - tb);  // the next block's steps (0: none)
    // 1. inferred transfers: u^n with NEIGHBORHOOD(tb), u^{n-1} with NEIGHBORHOOD(tb-1)
    jobs.clear();
    if (nchunks > 1 && !halos_ready) {
      ccl_range_mapper m;
      memset(&m, 0, sizeof(m));
      m.kind = CCL_MAP_NEIGHBORHOOD;
      for (int d = 0; d < dims; ++d) m.extent[d] = tb;
      st = exchange_jobs(nchunks, chunks, m, u_cur, esize, &jobs);
      if (st != CCL_OK) return st;
      if (tb > 1) {
        for (int d = 0; d < dims; ++d) m.extent[d] = tb - 1;
        st = exchange_jobs(nchunks, chunks, m, u_prev, esize, &jobs);
        if (st != CCL_OK) return st;
      }
      if (!jobs.empty()) {
        st = launch_copies(jobs.data(), static_cast<int32_t>(jobs.size()), stream);
        if (st != CCL_OK) return st;
      }
    }
    // 2. one launch advances all chunks tb steps
    for (int k = 0; k < nchunks; ++k) {
      WaveChunkPlan &P = plans[k];
      P.chunk = chunk_box(chunks[k]);
      P.domain = domain_box(chunks[k]);
      P.in_prev = field_of(u_prev[k]);
      P.in_cur = field_of(u_cur[k]);
      P.out_prev = in_place ? field_of(u_prev[k]) : field_of(w_prev[k]);
      P.out_cur = in_place ? field_of(u_prev[k]) : field_of(w_cur[k]);
      P.load_prev = intersect(box_of(u_prev[k].region), P.domain);
      P.load_cur = intersect(box_of(u_cur[k].region), P.domain);
    }
    bool pushed = false;
    if (can_push && next > 0)
      pushed = plan_pushes(nchunks, chunks, in_place ? u_prev : w_cur, in_place ? nullptr : w_prev,
                           next, plans.data());
    if (!pushed)
      for (int k = 0; k < nchunks; ++k) plans[k].npush = 0;
    if (dims == 2)
      st = launch_wave2d(dtype, tb, in_place, p->r2, p->tile_rows, plans.data(), nchunks,
                         stream, pushed ? &pushed : nullptr);
    else
      st = launch_wave3d(dtype, tb, in_place, p->r2, p->tile_rows, plans.data(), nchunks,
                         stream);
    if (st != CCL_OK) return st;
    halos_ready = pushed;
    // 3. rotate roles so u_cur names the newest level
    for (int k = 0; k < nchunks; ++k) {
      if (in_place) {
        std::swap(u_prev[k], u_cur[k]);
      } else {
        std::swap(u_prev[k], w_prev[k]);
        std::swap(u_cur[k], w_cur[k]);
      }
    }
    done += tb;
  }
  return CCL_OK;
}
