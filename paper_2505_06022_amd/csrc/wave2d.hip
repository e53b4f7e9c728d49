// 2D five-point leapfrog stencil over device-local chunks, T steps per pass.
//
// Work unit: one wave (64 lanes) owns a tile = a strip of 256 columns (four
// consecutive floats per lane, 16-byte loads) and a segment of output rows.
// The wave streams down the rows: at iteration i it loads row i of u^n and
// row i-1 of u^{n-1}, then computes level 2 at row i-1, level 3 at row i-2,
// ..., level T+1 at row i-T, keeping the last three rows of every level in
// registers.  North/south neighbours come from that register ring; west/east
// neighbours from the adjacent lane through DPP wave shifts (no LDS, no
// barriers).  A level-(k+1) value is only valid where its whole dependency
// cone was loaded, so strips overlap by 4*ceil(T/4) columns on each side and
// segments re-read T rows above and below; outputs are written only for the
// valid interior.  Every cell value is produced by the same float32
// expression, so results are bitwise independent of T, tiling and chunking.
//
// T == 1 runs in place: u^{n+1} overwrites u^{n-1}; each lane then reads
// u^{n-1} only at the cells it writes.  T > 1 writes u^{n+T-1} and u^{n+T}
// to a second buffer pair because neighbouring tiles still read the halo
// cells of the inputs.
#include <algorithm>
#include <cstring>

#include "ccl_internal.h"

namespace ccl {
namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kThreads = 64 * kWavesPerBlock;
constexpr int kMaxChunksPerLaunch = 16;
constexpr int kPrefetch = 3;

struct W2Chunk {
  const float *in_prev;
  const float *in_cur;
  float *out_prev;
  float *out_cur;
  int32_t ip_y0, ip_x0, ip_pitch;
  int32_t ic_y0, ic_x0, ic_pitch;
  int32_t op_y0, op_x0, op_pitch;
  int32_t oc_y0, oc_x0, oc_pitch;
  int32_t lp_y0, lp_y1, lp_x0, lp_x1;  // loadable box of in_prev
  int32_t lc_y0, lc_y1, lc_x0, lc_x1;  // loadable box of in_cur
  int32_t cy0, cy1, cx0, cx1;          // chunk (output) box
  int32_t xs0;                         // first column of strip 0
  int32_t nstrips;
  int32_t tile_begin;
};

struct W2Args {
  int32_t nchunks;
  int32_t total_tiles;
  int32_t tile_rows;
  int32_t gy0, gy1, gx0, gx1;  // domain: zero outside
  float r2;
  W2Chunk ch[kMaxChunksPerLaunch];
};

__device__ __forceinline__ float dpp_from_left(float v) {
  // lane l receives lane l-1's value (wave_shr:1); lane 0 receives 0
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float dpp_from_right(float v) {
  // lane l receives lane l+1's value (wave_shl:1); lane 63 receives 0
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}

// One cell: s = (N + S) + (W + E); lap = s - 4C; u+ = fma(r2, lap, 2C - P).
__device__ __forceinline__ float cell(float n, float s, float w, float e, float c, float p,
                                      float r2) {
  const float sum = (n + s) + (w + e);
  const float lap = sum - 4.0f * c;
  return fmaf(r2, lap, 2.0f * c - p);
}

__device__ __forceinline__ float4 step4(const float4 &n, const float4 &c, const float4 &s,
                                        const float4 &p, float r2) {
  const float left = dpp_from_left(c.w);
  const float right = dpp_from_right(c.x);
  float4 o;
  o.x = cell(n.x, s.x, left, c.y, c.x, p.x, r2);
  o.y = cell(n.y, s.y, c.x, c.z, c.y, p.y, r2);
  o.z = cell(n.z, s.z, c.y, c.w, c.z, p.z, r2);
  o.w = cell(n.w, s.w, c.z, right, c.w, p.w, r2);
  return o;
}

__device__ __forceinline__ float4 zero4() { return make_float4(0.f, 0.f, 0.f, 0.f); }

// Per-lane column mask of one field: which of the lane's four columns
// [xl, xl+4) lie in the loadable range [x0, x1).  Columns are grouped in
// aligned fours relative to the buffer, and a buffer's pitch is a multiple
// of 4 that covers its extent, so a group that meets [x0, x1) is always
// inside the allocated row.
struct Cols {
  bool any, m0, m1, m2, m3;
};

__device__ __forceinline__ Cols cols_of(int xl, int x0, int x1) {
  Cols c;
  c.m0 = xl + 0 >= x0 && xl + 0 < x1;
  c.m1 = xl + 1 >= x0 && xl + 1 < x1;
  c.m2 = xl + 2 >= x0 && xl + 2 < x1;
  c.m3 = xl + 3 >= x0 && xl + 3 < x1;
  c.any = c.m0 || c.m1 || c.m2 || c.m3;
  return c;
}

// Loads the lane's group of `row` (zero outside the loadable box).
__device__ __forceinline__ float4 load4(const float *base, int32_t by0, int32_t bx0,
                                        int32_t pitch, int row, int xl, int ly0, int ly1,
                                        const Cols &c) {
  float4 v = zero4();
  if (row < ly0 || row >= ly1) return v;  // wave-uniform
  if (c.any) v = *reinterpret_cast<const float4 *>(
                 base + static_cast<int64_t>(row - by0) * pitch + (xl - bx0));
  v.x = c.m0 ? v.x : 0.0f;
  v.y = c.m1 ? v.y : 0.0f;
  v.z = c.m2 ? v.z : 0.0f;
  v.w = c.m3 ? v.w : 0.0f;
  return v;
}

// Stores the lane's group of `row` where the output mask allows.  Partial
// groups occur only at a chunk's left or right edge; their other columns are
// halo cells of this chunk's own buffer that no wave writes during the
// launch, so they are read and written back unchanged (one 16-byte store).
__device__ __forceinline__ void store4(float *base, int32_t by0, int32_t bx0, int32_t pitch,
                                       int row, int xl, const Cols &c, const float4 &v) {
  if (!c.any) return;
  float4 *p = reinterpret_cast<float4 *>(base + static_cast<int64_t>(row - by0) * pitch +
                                         (xl - bx0));
  float4 w = v;
  if (!(c.m0 && c.m1 && c.m2 && c.m3)) {
    const float4 o = *p;
    w.x = c.m0 ? v.x : o.x;
    w.y = c.m1 ? v.y : o.y;
    w.z = c.m2 ? v.z : o.z;
    w.w = c.m3 ? v.w : o.w;
  }
  *p = w;
}

__device__ __forceinline__ float4 force_zero(float4 v, bool row_in, bool m0, bool m1, bool m2,
                                             bool m3) {
  v.x = (row_in && m0) ? v.x : 0.0f;
  v.y = (row_in && m1) ? v.y : 0.0f;
  v.z = (row_in && m2) ? v.z : 0.0f;
  v.w = (row_in && m3) ? v.w : 0.0f;
  return v;
}

// Maps a block index so that consecutive logical blocks land on the same
// XCD (blocks are dispatched to the 8 XCDs round-robin); neighbouring tiles
// then share an L2 for the rows and columns they both read.
__device__ __forceinline__ int xcd_block(int bid, int nblocks) {
  const int q = nblocks >> 3, r = nblocks & 7;
  const int xcd = bid & 7, idx = bid >> 3;
  return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + idx;
}

template <int T, bool IN_PLACE>
__global__ __launch_bounds__(kThreads) void wave2d_kernel(const W2Args a) {
  constexpr int A = 4 * ((T + 3) / 4);  // overlap columns per side
  constexpr int SW = 256 - 2 * A;       // output columns per strip
  const int lane = threadIdx.x & 63;
  const int tile = __builtin_amdgcn_readfirstlane(
      xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + (threadIdx.x >> 6));
  if (tile >= a.total_tiles) return;
  int c = 0;
  while (c + 1 < a.nchunks && tile >= a.ch[c + 1].tile_begin) ++c;
  const W2Chunk &C = a.ch[c];

  const int local = tile - C.tile_begin;
  const int seg = local / C.nstrips;
  const int strip = local - seg * C.nstrips;
  const int y0 = C.cy0 + seg * a.tile_rows;
  const int y1 = min(C.cy1, y0 + a.tile_rows);
  const int xs = C.xs0 + strip * SW;
  const int xl = xs + 4 * lane;
  const int vx0 = max(C.cx0, xs + A);
  const int vx1 = min(C.cx1, xs + A + SW);
  const float r2 = a.r2;

  const Cols dom = cols_of(xl, a.gx0, a.gx1);
  const Cols out = cols_of(xl, vx0, vx1);
  const Cols lc = cols_of(xl, C.lc_x0, C.lc_x1);
  // In place, u^{n-1} is read only where this lane writes.
  const int lpy0 = IN_PLACE ? max(C.lp_y0, y0) : C.lp_y0;
  const int lpy1 = IN_PLACE ? min(C.lp_y1, y1) : C.lp_y1;
  const Cols lp = cols_of(xl, IN_PLACE ? max(C.lp_x0, vx0) : C.lp_x0,
                          IN_PLACE ? min(C.lp_x1, vx1) : C.lp_x1);

  float4 ring[T][3];
#pragma unroll
  for (int k = 0; k < T; ++k) ring[k][0] = ring[k][1] = ring[k][2] = zero4();

  const int i0 = y0 - T;
  const int iend = y1 + T;  // exclusive
  float4 q1[kPrefetch], q0[kPrefetch];
#pragma unroll
  for (int u = 0; u < kPrefetch; ++u) {
    q1[u] = load4(C.in_cur, C.ic_y0, C.ic_x0, C.ic_pitch, i0 + u, xl, C.lc_y0, C.lc_y1, lc);
    q0[u] = load4(C.in_prev, C.ip_y0, C.ip_x0, C.ip_pitch, i0 + u - 1, xl, lpy0, lpy1, lp);
  }

  for (int base = i0; base < iend; base += kPrefetch) {
#pragma unroll
    for (int u = 0; u < kPrefetch; ++u) {
      const int i = base + u;
      const float4 v1 = q1[u];
      const float4 v0 = q0[u];
      q1[u] = load4(C.in_cur, C.ic_y0, C.ic_x0, C.ic_pitch, i + kPrefetch, xl, C.lc_y0, C.lc_y1,
                    lc);
      q0[u] = load4(C.in_prev, C.ip_y0, C.ip_x0, C.ip_pitch, i + kPrefetch - 1, xl, lpy0, lpy1,
                    lp);
      ring[0][0] = ring[0][1];
      ring[0][1] = ring[0][2];
      ring[0][2] = v1;
      float4 pv = v0;
#pragma unroll
      for (int k = 1; k <= T; ++k) {
        const int r = i - k;  // row of level k+1 computed now
        float4 nv = step4(ring[k - 1][0], ring[k - 1][1], ring[k - 1][2], pv, r2);
        nv = force_zero(nv, r >= a.gy0 && r < a.gy1, dom.m0, dom.m1, dom.m2, dom.m3);
        if (k < T) {
          pv = ring[k - 1][0];
          ring[k][0] = ring[k][1];
          ring[k][1] = ring[k][2];
          ring[k][2] = nv;
        } else if (r >= y0 && r < y1) {
          store4(C.out_cur, C.oc_y0, C.oc_x0, C.oc_pitch, r, xl, out, nv);
          if (!IN_PLACE)
            store4(C.out_prev, C.op_y0, C.op_x0, C.op_pitch, r, xl, out, ring[T - 1][1]);
        }
      }
    }
  }
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

int32_t wave2d_auto_rows(int32_t depth, int64_t rows, int64_t cols, int32_t nchunks) {
  // Aim at ~8 waves per SIMD (256 CUs x 4 SIMDs) while keeping the 2T-row
  // re-read per segment below ~1/8 of the segment.
  const int A = 4 * ((depth + 3) / 4);
  const int64_t strips = (cols + (256 - 2 * A) - 1) / (256 - 2 * A);
  const int64_t target_waves = 8192;
  int64_t r = (rows * strips + target_waves - 1) / target_waves;
  r = std::max<int64_t>(r, 16 * depth);
  r = std::max<int64_t>(r, 16);
  r = (r + 7) / 8 * 8;
  (void)nchunks;
  return static_cast<int32_t>(std::min<int64_t>(r, 1 << 20));
}

ccl_status launch_wave2d(int32_t depth, bool in_place, float r2, int32_t tile_rows,
                         const WaveChunkPlan *plans, int32_t nplans, hipStream_t stream) {
  const int A = 4 * ((depth + 3) / 4);
  const int SW = 256 - 2 * A;
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
    a.gy0 = static_cast<int32_t>(dom.lo[0]);
    a.gy1 = static_cast<int32_t>(dom.hi[0]);
    a.gx0 = static_cast<int32_t>(dom.lo[1]);
    a.gx1 = static_cast<int32_t>(dom.hi[1]);
    int64_t rows_max = 0, cols_max = 0;
    for (int k = 0; k < n; ++k) {
      const Box &cb = plans[first + k].chunk;
      rows_max = std::max<int64_t>(rows_max, cb.hi[0] - cb.lo[0]);
      cols_max = std::max<int64_t>(cols_max, cb.hi[1] - cb.lo[1]);
    }
    a.tile_rows = tile_rows > 0 ? tile_rows
                                : wave2d_auto_rows(depth, rows_max * n, cols_max, n);
    int64_t tiles = 0;
    for (int k = 0; k < n; ++k) {
      const WaveChunkPlan &P = plans[first + k];
      W2Chunk &C = a.ch[k];
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
      const int64_t segs = (P.chunk.hi[0] - P.chunk.lo[0] + a.tile_rows - 1) / a.tile_rows;
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
