// Internal declarations shared by the translation units of libccl.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "ccl.h"

namespace ccl {

// Bytes of one stored element of a ccl dtype (0 if unknown).
constexpr int dtype_bytes(int32_t dtype) {
  return dtype == CCL_DTYPE_F32 ? 4 : dtype == CCL_DTYPE_F64 ? 8
       : (dtype == CCL_DTYPE_BF16 || dtype == CCL_DTYPE_F16) ? 2 : 0;
}

// Elements a lane loads as one vector access (16 bytes of registers: four
// floats or two doubles; four 16-bit values widen to four floats).
constexpr int dtype_group(int32_t dtype) { return dtype == CCL_DTYPE_F64 ? 2 : 4; }

// Records a message for ccl_last_error() and returns `st`.
ccl_status fail(ccl_status st, const char *fmt, ...);
void clear_error();

inline ccl_status hip_check(hipError_t e, const char *what) {
  if (e == hipSuccess) return CCL_OK;
  return fail(CCL_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Half-open interval helpers on int64 boxes.
struct Box {
  int32_t dims = 0;
  int64_t lo[CCL_MAX_DIMS] = {0, 0, 0};
  int64_t hi[CCL_MAX_DIMS] = {0, 0, 0};
  bool empty() const {
    for (int d = 0; d < dims; ++d)
      if (hi[d] <= lo[d]) return true;
    return false;
  }
  int64_t volume() const {
    int64_t v = 1;
    for (int d = 0; d < dims; ++d) v *= (hi[d] > lo[d] ? hi[d] - lo[d] : 0);
    return v;
  }
};

Box box_of(const ccl_subrange &s);
Box chunk_box(const ccl_chunk &c);
Box domain_box(const ccl_chunk &c);
ccl_subrange subrange_of(const Box &b);
Box intersect(const Box &a, const Box &b);
bool contains(const Box &outer, const Box &inner);
Box grow(const Box &b, int64_t e);  // by e along every dimension

// Region of the buffer [0, buffer_range) that chunk `c` touches through `m`.
ccl_status region_box(const ccl_chunk &c, const ccl_range_mapper &m, const int64_t *buffer_range,
                      Box *out);
ccl_status check_chunks(int32_t nchunks, const ccl_chunk *chunks, int32_t dims);
ccl_status check_buffer(const ccl_chunk_buffer &b, int32_t dims, const char *what,
                        bool need_vec_align);

// Brackets one kernel launch with timing events when timing is enabled.
class TimedLaunch {
 public:
  TimedLaunch(int kind, hipStream_t s);
  ~TimedLaunch();
  TimedLaunch(const TimedLaunch &) = delete;
  TimedLaunch &operator=(const TimedLaunch &) = delete;

 private:
  int kind_;
  hipStream_t stream_;
  std::pair<hipEvent_t, hipEvent_t> ev_{};
  bool active_ = false;
};

// ---- halo copies (halo.hip) ----------------------------------------------
// One copy job: a box of units from src to dst, a unit being 4 bytes (or 2
// for 2-byte elements).  Strides and the contiguous extent in units.
struct CopyJob {
  const void *src;
  void *dst;
  int64_t src_pitch0, src_pitch1;  // units per step of dim 0 / dim 1
  int64_t dst_pitch0, dst_pitch1;
  int32_t n0, n1, n2;              // extents (dim 2 in units, contiguous)
  int32_t unit;                    // bytes per unit: 4 or 2
};
// Enqueues all jobs (any count; split into launches internally).
ccl_status launch_copies(const CopyJob *jobs, int32_t njobs, hipStream_t stream);
// Appends the copy jobs of every transfer that `mapper` infers among the
// chunk buffers (reader region ∩ owner chunk), validating both buffers.
ccl_status exchange_jobs(int32_t nchunks, const ccl_chunk *chunks, const ccl_range_mapper &mapper,
                         const ccl_chunk_buffer *bufs, int32_t elem_bytes,
                         std::vector<CopyJob> *jobs);

// ---- wave kernels --------------------------------------------------------
struct WaveField {      // one chunk buffer as the kernels see it
  void *base;
  int64_t off[CCL_MAX_DIMS];
  int64_t pitch[CCL_MAX_DIMS];
};

// Rows of a chunk's output that another chunk's next block reads: stored by
// the launch into that chunk's output buffers as well (2D, splits along
// rows).  [cr0, cr1) of u^{n+T} into `cur`, [pr0, pr1) of u^{n+T-1} into
// `prev` (empty ranges allowed).
struct PushPlan {
  WaveField cur, prev;
  int64_t cr0, cr1, pr0, pr1;
};
constexpr int kMaxPushPerChunk = 2;

struct WaveChunkPlan {  // host-side plan of one chunk for one block of steps
  Box chunk;
  Box domain;
  WaveField in_prev, in_cur, out_prev, out_cur;
  Box load_prev, load_cur;  // loadable index boxes (region of the buffer ∩ domain)
  int32_t npush = 0;
  PushPlan push[kMaxPushPerChunk];
};

// Rows (2D) or planes (3D) per tile when the caller leaves it to the
// library: every wave streams (rows + 2*halo) rows, rounded up to a whole
// number of its loop bodies of `granule` rows, and the launch runs in
// ceil(waves / slots) rounds of concurrently resident waves, so the rows are
// chosen to minimise rounds * streamed rows.  `waves_of(rows)` is the
// launch's wave count for a given rows value (non-increasing in rows).
template <class F>
int32_t plan_tile_rows(int64_t slots, int32_t halo, int32_t min_rows, int32_t max_rows,
                       F waves_of, int32_t granule = 1) {
  if (slots < 1) slots = 1;
  if (max_rows < min_rows) max_rows = min_rows;
  int32_t best = max_rows;
  double best_cost = 1e300;
  for (int64_t m = 1; m <= 64; ++m) {
    // smallest rows whose wave count fits in m rounds
    int32_t lo = min_rows, hi = max_rows;
    if (waves_of(hi) > m * slots) continue;
    while (lo < hi) {
      const int32_t mid = lo + (hi - lo) / 2;
      if (waves_of(mid) <= m * slots)
        hi = mid;
      else
        lo = mid + 1;
    }
    const int64_t w = waves_of(lo);
    const double rounds = static_cast<double>((w + slots - 1) / slots);
    const int64_t streamed = (lo + 2 * static_cast<int64_t>(halo) + granule - 1) / granule * granule;
    const double cost = rounds * static_cast<double>(streamed);
    if (cost < best_cost - 1e-9) {
      best_cost = cost;
      best = lo;
    }
    if (lo == min_rows) break;
  }
  return best;
}

int32_t wave2d_plan_rows(int64_t ny, int64_t nx, int32_t K, int32_t T);
// Waves of the depth-T kernel the device holds at once (occupancy API; a
// fixed guess where no device answers).
int64_t wave2d_slots(int32_t T);
int64_t wave3d_slots(int32_t T);
int64_t wave3d_tb_wave_slots(int32_t T);
int32_t wave3d_plan_planes(int64_t nz, int64_t ny, int64_t nx, int32_t K, int32_t T);
int32_t wave3d_tb_plan_planes(int64_t nz, int64_t ny, int64_t nx, int32_t K, int32_t T);
// Output columns and rows of one block's patch, and waves per block, of the
// depth-T (2..8) 3D kernel.
void wave3d_tb_geometry(int32_t T, int32_t *out_cols, int32_t *out_rows, int32_t *waves);

// dtype: CCL_DTYPE_* of every buffer; r2 as given (rounded to float for
// float arithmetic).
// `pushed` (may be NULL): set to whether every push the plans ask for was
// made; if any cannot be (count, alignment), none is and it is false.
ccl_status launch_wave2d(int32_t dtype, int32_t depth, bool in_place, double r2,
                         int32_t tile_rows, const WaveChunkPlan *plans, int32_t nplans,
                         hipStream_t stream, bool *pushed = nullptr);
ccl_status launch_wave3d(int32_t dtype, int32_t depth, bool in_place, double r2,
                         int32_t tile_rows, const WaveChunkPlan *plans, int32_t nplans,
                         hipStream_t stream);
// Depth T in 2..8, out of place (u^{n+T-1}, u^{n+T} to out_prev, out_cur).
ccl_status launch_wave3d_tb(int32_t dtype, int32_t T, double r2, int32_t tile_planes,
                            const WaveChunkPlan *plans, int32_t nplans, hipStream_t stream);

}  // namespace ccl
