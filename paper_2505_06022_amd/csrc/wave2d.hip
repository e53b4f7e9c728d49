// 2D five-point leapfrog stencil over device-local chunks, T steps per
// launch.  The per-tile device code (row streaming with register rings and
// DPP neighbour exchange) is in wave2d_tile.h; this file maps the launch's
// waves onto the tiles of all chunks and plans the launch on the host.
#include <algorithm>
#include <cstring>

#include "ccl_internal.h"
#include "wave2d_tile.h"

namespace ccl {
namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kThreads = 64 * kWavesPerBlock;
constexpr int kMaxChunksPerLaunch = 16;
constexpr int kMaxPushPerLaunch = 16;

struct W2Args {
  int32_t nchunks;
  int32_t total_tiles;
  int32_t tile_rows;
  w2::Domain dom;
  float r2f;   // r2 rounded to float (float arithmetic)
  double r2d;  // r2 as given (double arithmetic)
  w2::Chunk ch[kMaxChunksPerLaunch];
  w2::Push push[kMaxPushPerLaunch];
};

template <class F>
__device__ __forceinline__ F r2_of(const W2Args &a);
template <>
__device__ __forceinline__ float r2_of<float>(const W2Args &a) { return a.r2f; }
template <>
__device__ __forceinline__ double r2_of<double>(const W2Args &a) { return a.r2d; }

template <class PR, int T, bool IN_PLACE>
__global__ __launch_bounds__(kThreads) void wave2d_kernel(const W2Args a) {
  const int lane = threadIdx.x & 63;
  const int tile = __builtin_amdgcn_readfirstlane(
      w2::xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + (threadIdx.x >> 6));
  if (tile >= a.total_tiles) return;
  int c = 0;
  while (c + 1 < a.nchunks && tile >= a.ch[c + 1].tile_begin) ++c;
  const w2::Chunk &C = a.ch[c];
  const int local = tile - C.tile_begin;
  const int seg = local / C.nstrips;
  const int strip = local - seg * C.nstrips;
  w2::PushSet ps;
  ps.n = C.push_end - C.push_begin;
#pragma unroll
  for (int p = 0; p < w2::kMaxPush; ++p) ps.p[p] = a.push[min(C.push_begin + p, kMaxPushPerLaunch - 1)];
  w2::tile<PR, T, IN_PLACE>(C, a.dom, r2_of<typename PR::F>(a), a.tile_rows, seg, strip, lane,
                            w2::overlap(T, PR::NV), ps);
}

template <class PR, int T, bool IP>
ccl_status launch_t(const W2Args &a, int blocks, hipStream_t s) {
  TimedLaunch tl(CCL_KERNEL_STENCIL, s);
  hipLaunchKernelGGL((wave2d_kernel<PR, T, IP>), dim3(blocks), dim3(kThreads), 0, s, a);
  return hip_check(hipGetLastError(), "wave2d_kernel launch");
}

template <class PR>
ccl_status launch_depth(int T, bool in_place, const W2Args &a, int blocks, hipStream_t s) {
  if (in_place) {
    if (T != 1) return fail(CCL_E_INVALID, "in-place update needs T == 1");
    return launch_t<PR, 1, true>(a, blocks, s);
  }
  switch (T) {
    case 1: return launch_t<PR, 1, false>(a, blocks, s);
    case 2: return launch_t<PR, 2, false>(a, blocks, s);
    case 3: return launch_t<PR, 3, false>(a, blocks, s);
    case 4: return launch_t<PR, 4, false>(a, blocks, s);
    case 5: return launch_t<PR, 5, false>(a, blocks, s);
    case 6: return launch_t<PR, 6, false>(a, blocks, s);
    case 7: return launch_t<PR, 7, false>(a, blocks, s);
    case 8: return launch_t<PR, 8, false>(a, blocks, s);
    default: return fail(CCL_E_INVALID, "temporal depth %d not in 1..8", T);
  }
}

ccl_status launch_dtype(int32_t dtype, int T, bool in_place, const W2Args &a, int blocks,
                        hipStream_t s) {
  switch (dtype) {
    case CCL_DTYPE_F32: return launch_depth<P32>(T, in_place, a, blocks, s);
    case CCL_DTYPE_F64: return launch_depth<P64>(T, in_place, a, blocks, s);
    case CCL_DTYPE_BF16: return launch_depth<PB16>(T, in_place, a, blocks, s);
    case CCL_DTYPE_F16: return launch_depth<PH16>(T, in_place, a, blocks, s);
    default: return fail(CCL_E_INVALID, "unknown dtype %d", dtype);
  }
}

template <class PR>
const void *kernel_ptr(int T, bool in_place) {
  if (in_place) return reinterpret_cast<const void *>(&wave2d_kernel<PR, 1, true>);
  switch (T) {
    case 1: return reinterpret_cast<const void *>(&wave2d_kernel<PR, 1, false>);
    case 2: return reinterpret_cast<const void *>(&wave2d_kernel<PR, 2, false>);
    case 3: return reinterpret_cast<const void *>(&wave2d_kernel<PR, 3, false>);
    case 4: return reinterpret_cast<const void *>(&wave2d_kernel<PR, 4, false>);
    case 5: return reinterpret_cast<const void *>(&wave2d_kernel<PR, 5, false>);
    case 6: return reinterpret_cast<const void *>(&wave2d_kernel<PR, 6, false>);
    case 7: return reinterpret_cast<const void *>(&wave2d_kernel<PR, 7, false>);
    default: return reinterpret_cast<const void *>(&wave2d_kernel<PR, 8, false>);
  }
}

const void *kernel_for(int32_t dtype, int T, bool in_place) {
  switch (dtype) {
    case CCL_DTYPE_F64: return kernel_ptr<P64>(T, in_place);
    case CCL_DTYPE_BF16: return kernel_ptr<PB16>(T, in_place);
    case CCL_DTYPE_F16: return kernel_ptr<PH16>(T, in_place);
    default: return kernel_ptr<P32>(T, in_place);
  }
}

bool fits_i32(int64_t v) { return v >= INT32_MIN && v <= INT32_MAX; }

// Rows per loop body of the kernel a launch of this type and mode runs.
int32_t body_rows(int32_t dtype, bool in_place) {
  switch (dtype) {
    case CCL_DTYPE_F64: return w2::unroll_of<P64>(in_place);
    case CCL_DTYPE_BF16: return w2::unroll_of<PB16>(in_place);
    case CCL_DTYPE_F16: return w2::unroll_of<PH16>(in_place);
    default: return w2::unroll_of<P32>(in_place);
  }
}

}  // namespace

// Concurrent waves the device holds for the depth-T kernel (cached).
static int64_t wave_slots(int T, bool in_place, int32_t dtype = CCL_DTYPE_F32) {
  static int64_t cache[4][2][CCL_MAX_DEPTH + 1] = {};
  if (dtype < 0 || dtype > 3) dtype = CCL_DTYPE_F32;
  int64_t &c = cache[dtype][in_place ? 1 : 0][T];
  if (c > 0) return c;
  const void *fn = kernel_for(dtype, T, in_place);
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads, 0) != hipSuccess ||
      per_cu < 1) {
    return 1024;  // planning only; any positive value gives a valid launch
  }
  c = static_cast<int64_t>(cus) * per_cu * kWavesPerBlock;
  return c;
}

int64_t wave2d_slots(int32_t T) { return wave_slots(T, T == 1); }

// The rows the launcher would pick for a domain split into K row chunks
// (buffers starting at the domain's first column).
int32_t wave2d_plan_rows(int64_t ny, int64_t nx, int32_t K, int32_t T) {
  const int SW = w2::strip_width(T);
  const int64_t nstrips = (nx + SW - 1) / SW;
  int64_t rows_max = 0;
  for (int k = 0; k < K; ++k) rows_max = std::max<int64_t>(rows_max, (k + 1) * ny / K - k * ny / K);
  auto waves_of = [&](int32_t r) {
    int64_t w = 0;
    for (int k = 0; k < K; ++k) {
      const int64_t rows = (k + 1) * ny / K - k * ny / K;
      w += ((rows + r - 1) / r) * nstrips;
    }
    return w;
  };
  return plan_tile_rows(wave_slots(T, T == 1), T, std::max(8, T),
                        static_cast<int32_t>(std::max<int64_t>(rows_max, 8)), waves_of,
                        w2::unroll_of<P32>(T == 1));
}

ccl_status launch_wave2d(int32_t dtype, int32_t depth, bool in_place, double r2,
                         int32_t tile_rows, const WaveChunkPlan *plans, int32_t nplans,
                         hipStream_t stream, bool *pushed) {
  bool all_pushed = true;  // every push the plans ask for is encoded
  const int NV = dtype_group(dtype);
  const int esize = dtype_bytes(dtype);
  if (esize == 0) return fail(CCL_E_INVALID, "unknown dtype %d", dtype);
  const int A = w2::overlap(depth, NV);
  const int SW = w2::strip_width(depth, NV);
  for (int first = 0; first < nplans; first += kMaxChunksPerLaunch) {
    const int n = std::min(kMaxChunksPerLaunch, nplans - first);
    W2Args a;
    memset(&a, 0, sizeof(a));
    a.nchunks = n;
    a.r2f = static_cast<float>(r2);
    a.r2d = r2;
    const Box &dom = plans[first].domain;
    if (!fits_i32(dom.lo[0] - 64) || !fits_i32(dom.hi[0] + 64) || !fits_i32(dom.lo[1] - 512) ||
        !fits_i32(dom.hi[1] + 512))
      return fail(CCL_E_RANGE, "2D indices must fit in int32");
    a.dom.gy0 = static_cast<int32_t>(dom.lo[0]);
    a.dom.gy1 = static_cast<int32_t>(dom.hi[0]);
    a.dom.gx0 = static_cast<int32_t>(dom.lo[1]);
    a.dom.gx1 = static_cast<int32_t>(dom.hi[1]);
    int64_t rows_max = 0;
    for (int k = 0; k < n; ++k) {
      const Box &cb = plans[first + k].chunk;
      rows_max = std::max<int64_t>(rows_max, cb.hi[0] - cb.lo[0]);
    }
    for (int k = 0; k < n; ++k) {
      const WaveChunkPlan &P = plans[first + k];
      w2::Chunk &C = a.ch[k];
      C.in_prev = P.in_prev.base;
      C.in_cur = P.in_cur.base;
      C.out_prev = P.out_prev.base;
      C.out_cur = P.out_cur.base;
      const WaveField *f[4] = {&P.in_prev, &P.in_cur, &P.out_prev, &P.out_cur};
      int32_t *dst[4] = {&C.ip_y0, &C.ic_y0, &C.op_y0, &C.oc_y0};
      for (int b = 0; b < 4; ++b) {
        if (!fits_i32(f[b]->off[0]) || !fits_i32(f[b]->off[1]) || !fits_i32(f[b]->pitch[0]))
          return fail(CCL_E_RANGE, "2D buffer geometry must fit in int32");
        dst[b][0] = static_cast<int32_t>(f[b]->off[0]);
        dst[b][1] = static_cast<int32_t>(f[b]->off[1]);
        dst[b][2] = static_cast<int32_t>(f[b]->pitch[0]);
      }
      C.lp_y0 = static_cast<int32_t>(P.load_prev.lo[0]);
      C.lp_y1 = static_cast<int32_t>(P.load_prev.hi[0]);
      C.lp_x0 = static_cast<int32_t>(P.load_prev.lo[1]);
      C.lp_x1 = static_cast<int32_t>(P.load_prev.hi[1]);
      C.lc_y0 = static_cast<int32_t>(P.load_cur.lo[0]);
      C.lc_y1 = static_cast<int32_t>(P.load_cur.hi[0]);
      C.lc_x0 = static_cast<int32_t>(P.load_cur.lo[1]);
      C.lc_x1 = static_cast<int32_t>(P.load_cur.hi[1]);
      C.cy0 = static_cast<int32_t>(P.chunk.lo[0]);
      C.cy1 = static_cast<int32_t>(P.chunk.hi[0]);
      C.cx0 = static_cast<int32_t>(P.chunk.lo[1]);
      C.cx1 = static_cast<int32_t>(P.chunk.hi[1]);
      // strip 0 starts A columns left of the chunk, aligned down to a
      // multiple of NV relative to the u^n buffer so each lane's group is
      // one aligned vector access
      int64_t xs0 = P.chunk.lo[1] - A;
      int64_t rel = xs0 - P.in_cur.off[1];
      int64_t mis = ((rel % NV) + NV) % NV;
      xs0 -= mis;
      C.xs0 = static_cast<int32_t>(xs0);
      const int64_t width = P.chunk.hi[1] - (xs0 + A);
      C.nstrips = static_cast<int32_t>((width + SW - 1) / SW);
      const uintptr_t amask = static_cast<uintptr_t>(NV * esize - 1);
      for (int b = 0; b < 4; ++b) {
        const int64_t r = xs0 - f[b]->off[1];
        if ((((r % NV) + NV) % NV) != 0 || (f[b]->pitch[0] % NV) != 0 ||
            (reinterpret_cast<uintptr_t>(f[b]->base) & amask) != 0)
          return fail(CCL_E_INVALID,
                      "chunk %d: buffers must be %d-byte aligned, with pitch a multiple of %d and "
                      "the same region column offset modulo %d", first + k, NV * esize, NV, NV);
      }
      // halo pushes: the target buffers must hold the rows and the chunk's
      // columns and take the strips' groups at aligned boundaries
      C.push_begin = C.push_end = 0;
      for (int q = 0; q < P.npush && all_pushed; ++q) {
        const PushPlan &Q = P.push[q];
        const WaveField *tf[2] = {&Q.cur, &Q.prev};
        const int64_t rows[2][2] = {{Q.cr0, Q.cr1}, {Q.pr0, Q.pr1}};
        for (int b = 0; b < 2; ++b) {
          if (rows[b][1] <= rows[b][0]) continue;
          const int64_t r = xs0 - tf[b]->off[1];
          all_pushed = all_pushed && tf[b]->base && (((r % NV) + NV) % NV) == 0 &&
                       (tf[b]->pitch[0] % NV) == 0 &&
                       (reinterpret_cast<uintptr_t>(tf[b]->base) & amask) == 0 &&
                       fits_i32(tf[b]->off[0]) && fits_i32(tf[b]->off[1]) &&
                       fits_i32(tf[b]->pitch[0]);
        }
      }
    }
    // encode the pushes of this launch's chunks (all or none)
    int32_t npush = 0;
    for (int k = 0; k < n && all_pushed; ++k) {
      const WaveChunkPlan &P = plans[first + k];
      w2::Chunk &C = a.ch[k];
      C.push_begin = npush;
      if (P.npush > w2::kMaxPush) all_pushed = false;
      for (int q = 0; q < P.npush && all_pushed; ++q) {
        if (npush == kMaxPushPerLaunch) {
          all_pushed = false;
          break;
        }
        const PushPlan &Q = P.push[q];
        w2::Push &W = a.push[npush++];
        W.cur = Q.cur.base;
        W.prev = Q.prev.base;
        W.cur_y0 = static_cast<int32_t>(Q.cur.off[0]);
        W.cur_x0 = static_cast<int32_t>(Q.cur.off[1]);
        W.cur_pitch = static_cast<int32_t>(Q.cur.pitch[0]);
        W.prev_y0 = static_cast<int32_t>(Q.prev.off[0]);
        W.prev_x0 = static_cast<int32_t>(Q.prev.off[1]);
        W.prev_pitch = static_cast<int32_t>(Q.prev.pitch[0]);
        W.cr0 = static_cast<int32_t>(Q.cr0);
        W.cr1 = static_cast<int32_t>(std::max(Q.cr0, Q.cr1));
        W.pr0 = static_cast<int32_t>(Q.pr0);
        W.pr1 = static_cast<int32_t>(std::max(Q.pr0, Q.pr1));
      }
      C.push_end = npush;
    }
    if (!all_pushed)
      for (int k = 0; k < n; ++k) a.ch[k].push_begin = a.ch[k].push_end = 0;
    auto waves_of = [&](int32_t r) {
      int64_t w = 0;
      for (int k = 0; k < n; ++k)
        w += ((a.ch[k].cy1 - a.ch[k].cy0 + r - 1) / r) * static_cast<int64_t>(a.ch[k].nstrips);
      return w;
    };
    a.tile_rows = tile_rows > 0
                      ? tile_rows
                      : plan_tile_rows(wave_slots(depth, in_place, dtype), depth, std::max(8, depth),
                                       static_cast<int32_t>(std::max<int64_t>(rows_max, 8)),
                                       waves_of, body_rows(dtype, in_place));
    int64_t tiles = 0;
    for (int k = 0; k < n; ++k) {
      w2::Chunk &C = a.ch[k];
      const int64_t segs = (C.cy1 - C.cy0 + a.tile_rows - 1) / a.tile_rows;
      if (!fits_i32(tiles)) return fail(CCL_E_RANGE, "too many tiles");
      C.tile_begin = static_cast<int32_t>(tiles);
      tiles += segs * C.nstrips;
    }
    if (tiles > INT32_MAX / 2) return fail(CCL_E_RANGE, "too many tiles");
    a.total_tiles = static_cast<int32_t>(tiles);
    const int blocks = static_cast<int>((tiles + kWavesPerBlock - 1) / kWavesPerBlock);
    if (blocks == 0) continue;
    ccl_status st = launch_dtype(dtype, depth, in_place, a, blocks, stream);
    if (st != CCL_OK) return st;
  }
  if (pushed) *pushed = all_pushed;
  return CCL_OK;
}

}  // namespace ccl
