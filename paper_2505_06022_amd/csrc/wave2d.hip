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

struct W2Args {
  int32_t nchunks;
  int32_t total_tiles;
  int32_t tile_rows;
  w2::Domain dom;
  float r2;
  w2::Chunk ch[kMaxChunksPerLaunch];
};

template <int T, bool IN_PLACE>
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
  w2::tile<T, IN_PLACE>(C, a.dom, a.r2, a.tile_rows, seg, strip, lane, w2::overlap(T));
}

template <int T, bool IP>
ccl_status launch_t(const W2Args &a, int blocks, hipStream_t s) {
  TimedLaunch tl(CCL_KERNEL_STENCIL, s);
  hipLaunchKernelGGL((wave2d_kernel<T, IP>), dim3(blocks), dim3(kThreads), 0, s, a);
  return hip_check(hipGetLastError(), "wave2d_kernel launch");
}

ccl_status launch_depth(int T, bool in_place, const W2Args &a, int blocks, hipStream_t s) {
  if (in_place) {
    if (T != 1) return fail(CCL_E_INVALID, "in-place update needs T == 1");
    return launch_t<1, true>(a, blocks, s);
  }
  switch (T) {
    case 1: return launch_t<1, false>(a, blocks, s);
    case 2: return launch_t<2, false>(a, blocks, s);
    case 3: return launch_t<3, false>(a, blocks, s);
    case 4: return launch_t<4, false>(a, blocks, s);
    case 5: return launch_t<5, false>(a, blocks, s);
    case 6: return launch_t<6, false>(a, blocks, s);
    case 7: return launch_t<7, false>(a, blocks, s);
    case 8: return launch_t<8, false>(a, blocks, s);
    default: return fail(CCL_E_INVALID, "temporal depth %d not in 1..8", T);
  }
}

bool fits_i32(int64_t v) { return v >= INT32_MIN && v <= INT32_MAX; }

}  // namespace

// Concurrent waves the device holds for the depth-T kernel (cached).
static int64_t wave_slots(int T, bool in_place) {
  static int64_t cache[2][CCL_MAX_DEPTH + 1] = {};
  int64_t &c = cache[in_place ? 1 : 0][T];
  if (c > 0) return c;
  const void *fn = nullptr;
  switch (in_place ? 0 : T) {
    case 0: fn = reinterpret_cast<const void *>(&wave2d_kernel<1, true>); break;
    case 1: fn = reinterpret_cast<const void *>(&wave2d_kernel<1, false>); break;
    case 2: fn = reinterpret_cast<const void *>(&wave2d_kernel<2, false>); break;
    case 3: fn = reinterpret_cast<const void *>(&wave2d_kernel<3, false>); break;
    case 4: fn = reinterpret_cast<const void *>(&wave2d_kernel<4, false>); break;
    case 5: fn = reinterpret_cast<const void *>(&wave2d_kernel<5, false>); break;
    case 6: fn = reinterpret_cast<const void *>(&wave2d_kernel<6, false>); break;
    case 7: fn = reinterpret_cast<const void *>(&wave2d_kernel<7, false>); break;
    default: fn = reinterpret_cast<const void *>(&wave2d_kernel<8, false>); break;
  }
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
                        static_cast<int32_t>(std::max<int64_t>(rows_max, 8)), waves_of);
}

ccl_status launch_wave2d(int32_t depth, bool in_place, float r2, int32_t tile_rows,
                         const WaveChunkPlan *plans, int32_t nplans, hipStream_t stream) {
  const int A = w2::overlap(depth);
  const int SW = w2::strip_width(depth);
  for (int first = 0; first < nplans; first += kMaxChunksPerLaunch) {
    const int n = std::min(kMaxChunksPerLaunch, nplans - first);
    W2Args a;
    memset(&a, 0, sizeof(a));
    a.nchunks = n;
    a.r2 = r2;
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
      // multiple of 4 relative to the u^n buffer so its loads are 16-byte
      int64_t xs0 = P.chunk.lo[1] - A;
      int64_t rel = xs0 - P.in_cur.off[1];
      int64_t mis = ((rel % 4) + 4) % 4;
      xs0 -= mis;
      C.xs0 = static_cast<int32_t>(xs0);
      const int64_t width = P.chunk.hi[1] - (xs0 + A);
      C.nstrips = static_cast<int32_t>((width + SW - 1) / SW);
      for (int b = 0; b < 4; ++b) {
        const int64_t r = xs0 - f[b]->off[1];
        if ((((r % 4) + 4) % 4) != 0 || (f[b]->pitch[0] % 4) != 0 ||
            (reinterpret_cast<uintptr_t>(f[b]->base) & 15u) != 0)
          return fail(CCL_E_INVALID,
                      "chunk %d: buffers must be 16-byte aligned, with pitch a multiple of 4 and "
                      "the same region column offset modulo 4", first + k);
      }
    }
    auto waves_of = [&](int32_t r) {
      int64_t w = 0;
      for (int k = 0; k < n; ++k)
        w += ((a.ch[k].cy1 - a.ch[k].cy0 + r - 1) / r) * static_cast<int64_t>(a.ch[k].nstrips);
      return w;
    };
    a.tile_rows = tile_rows > 0
                      ? tile_rows
                      : plan_tile_rows(wave_slots(depth, in_place), depth, std::max(8, depth),
                                       static_cast<int32_t>(std::max<int64_t>(rows_max, 8)),
                                       waves_of);
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
    ccl_status st = launch_depth(depth, in_place, a, blocks, stream);
    if (st != CCL_OK) return st;
  }
  return CCL_OK;
}

}  // namespace ccl
