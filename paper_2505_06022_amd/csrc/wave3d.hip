// 3D seven-point leapfrog stencil over device-local chunks (one step per pass).
//
// Work unit: one wave owns a tile of 256 columns (four floats per lane) by
// R rows and streams along z through a segment of planes.  At iteration i it
// loads plane i of u^n for its R rows (the newest entry of a three-plane
// register ring), the two rows just outside its row block and the two
// columns just outside its strip (needed when plane i becomes the centre
// plane), and u^{n-1} of plane i-1; it then updates plane i-1 in place.
// z-neighbours come from the ring, y-neighbours from the lane's own rows or
// the halo rows, x-neighbours from the adjacent lane through DPP wave
// shifts, with the strip's two outer columns loaded by lanes 0 and 63.
#include <algorithm>
#include <cstring>

#include "ccl_internal.h"
#include "wave3d_cell.h"

namespace ccl {
namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kThreads = 64 * kWavesPerBlock;
constexpr int kMaxChunksPerLaunch = 16;
#ifndef CCL_W3_ROWS
#define CCL_W3_ROWS 4
#endif
constexpr int kRows = CCL_W3_ROWS;  // rows per wave tile

struct W3Chunk {
  const float *in_cur;
  float *io_prev;  // u^{n-1} in, u^{n+1} out
  int32_t ic_z0, ic_y0, ic_x0;
  int32_t ip_z0, ip_y0, ip_x0;
  int64_t ic_pz, ic_py;  // element strides of dims 0 and 1
  int64_t ip_pz, ip_py;
  int32_t lc_z0, lc_z1, lc_y0, lc_y1, lc_x0, lc_x1;  // loadable box of u^n
  int32_t cz0, cz1, cy0, cy1, cx0, cx1;              // chunk box
  int32_t xs0;                                       // first column of strip 0
  int32_t nstrips, nrowblk;
  int32_t tile_begin;
};

struct W3Args {
  int32_t nchunks;
  int32_t total_tiles;
  int32_t tile_planes;
  float r2;
  W3Chunk ch[kMaxChunksPerLaunch];
};

__device__ __forceinline__ float dpp_from_left(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float dpp_from_right(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}

__device__ __forceinline__ float4 zero4() { return make_float4(0.f, 0.f, 0.f, 0.f); }

struct Plane {
  float4 v[kRows];
};

// Which of the lane's four columns [xl, xl+4) lie in [x0, x1).  Groups are
// aligned fours relative to the buffer and pitches are multiples of 4 that
// cover the extent, so a group meeting [x0, x1) lies inside its row.
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

__device__ __forceinline__ float4 ld4(const float *base, int64_t pz, int64_t py, int z0, int y0,
                                      int x0, int z, int y, int xl, int lz0, int lz1, int ly0,
                                      int ly1, const Cols &c) {
  float4 v = zero4();
  if (z < lz0 || z >= lz1 || y < ly0 || y >= ly1) return v;  // wave-uniform
  if (c.any)
    v = *reinterpret_cast<const float4 *>(base + static_cast<int64_t>(z - z0) * pz +
                                          static_cast<int64_t>(y - y0) * py + (xl - x0));
  if (c.m0 && c.m1 && c.m2 && c.m3) return v;  // folds away when all are known true
  v.x = c.m0 ? v.x : 0.0f;
  v.y = c.m1 ? v.y : 0.0f;
  v.z = c.m2 ? v.z : 0.0f;
  v.w = c.m3 ? v.w : 0.0f;
  return v;
}

__device__ __forceinline__ int xcd_block(int bid, int nblocks) {
  const int q = nblocks >> 3, r = nblocks & 7;
  const int xcd = bid & 7, idx = bid >> 3;
  return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + idx;
}

// XIN: the strip's 256 columns lie inside the loadable and the output
// column ranges (every strip of a domain whose width is a multiple of 256),
// so loads and stores need no per-element column masks.
template <bool XIN>
__global__ __launch_bounds__(kThreads) void wave3d_kernel(const W3Args a) {
  const int lane = threadIdx.x & 63;
  const int tile = __builtin_amdgcn_readfirstlane(
      xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + (threadIdx.x >> 6));
  if (tile >= a.total_tiles) return;
  int c = 0;
  while (c + 1 < a.nchunks && tile >= a.ch[c + 1].tile_begin) ++c;
  const W3Chunk C = a.ch[c];  // in registers: not reloaded after stores

  // tile order: strip fastest, then row block, then z segment
  int local = tile - C.tile_begin;
  const int per_seg = C.nstrips * C.nrowblk;
  const int seg = local / per_seg;
  local -= seg * per_seg;
  const int rb = local / C.nstrips;
  const int strip = local - rb * C.nstrips;
  const int z0 = C.cz0 + seg * a.tile_planes;
  const int z1 = min(C.cz1, z0 + a.tile_planes);
  const int yb = C.cy0 + rb * kRows;
  const int xs = C.xs0 + strip * 256;
  const int xl = xs + 4 * lane;
  const float r2 = a.r2;

  // u^{n-1} is read (and written) only inside this tile's own output cells
  const int oy1 = min(C.cy1, yb + kRows);
  const Cols out = XIN ? Cols{true, true, true, true, true} : cols_of(xl, C.cx0, C.cx1);
  const Cols lc = XIN ? Cols{true, true, true, true, true} : cols_of(xl, C.lc_x0, C.lc_x1);
  const int edge_x = lane == 0 ? xs - 1 : xs + 256;
  const bool edge_lane = lane == 0 || lane == 63;

  Plane zm, zc, zp;  // ring: planes r-1, r, r+1 (r = centre)
  float4 hlo_c, hhi_c, hlo_n, hhi_n;  // halo rows of the centre / newest plane
  float ed_c[kRows], ed_n[kRows];     // outer columns of the centre / newest plane
#pragma unroll
  for (int j = 0; j < kRows; ++j) {
    zm.v[j] = zc.v[j] = zp.v[j] = zero4();
    ed_c[j] = ed_n[j] = 0.0f;
  }
  hlo_c = hhi_c = hlo_n = hhi_n = zero4();

  auto load_plane = [&](int z, Plane &pl, float4 &hlo, float4 &hhi, float *ed) {
#pragma unroll
    for (int j = 0; j < kRows; ++j)
      pl.v[j] = ld4(C.in_cur, C.ic_pz, C.ic_py, C.ic_z0, C.ic_y0, C.ic_x0, z, yb + j, xl, C.lc_z0,
                    C.lc_z1, C.lc_y0, C.lc_y1, lc);
    hlo = ld4(C.in_cur, C.ic_pz, C.ic_py, C.ic_z0, C.ic_y0, C.ic_x0, z, yb - 1, xl, C.lc_z0, C.lc_z1,
              C.lc_y0, C.lc_y1, lc);
    hhi = ld4(C.in_cur, C.ic_pz, C.ic_py, C.ic_z0, C.ic_y0, C.ic_x0, z, yb + kRows, xl, C.lc_z0,
              C.lc_z1, C.lc_y0, C.lc_y1, lc);
    const bool zin = z >= C.lc_z0 && z < C.lc_z1;
    const bool xin = edge_x >= C.lc_x0 && edge_x < C.lc_x1;
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      const int y = yb + j;
      float e = 0.0f;
      if (edge_lane && zin && xin && y >= C.lc_y0 && y < C.lc_y1)
        e = C.in_cur[static_cast<int64_t>(z - C.ic_z0) * C.ic_pz +
                     static_cast<int64_t>(y - C.ic_y0) * C.ic_py + (edge_x - C.ic_x0)];
      ed[j] = e;
    }
  };

  auto load_prev = [&](int z, float4 *pv) {
#pragma unroll
    for (int j = 0; j < kRows; ++j)
      pv[j] = ld4(C.io_prev, C.ip_pz, C.ip_py, C.ip_z0, C.ip_y0, C.ip_x0, z, yb + j, xl, z0, z1,
                  yb, oy1, out);
  };

  const int i0 = z0 - 1;
  // prime: plane z0-1 becomes the centre plane after the first shift
  load_plane(i0, zp, hlo_n, hhi_n, ed_n);
  Plane pn;
  float4 plo, phi;
  float ped[kRows];
  load_plane(i0 + 1, pn, plo, phi, ped);
  float4 pv[kRows], pvn[kRows];
  load_prev(i0, pvn);

  for (int i = i0 + 1; i <= z1; ++i) {
    // shift ring: newest becomes plane i
    zm = zc;
    zc = zp;
    zp = pn;
    hlo_c = hlo_n;
    hhi_c = hhi_n;
    hlo_n = plo;
    hhi_n = phi;
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      ed_c[j] = ed_n[j];
      ed_n[j] = ped[j];
      pv[j] = pvn[j];
    }
    const int r = i - 1;  // centre plane updated now
    // prefetch: u^{n-1} of plane i (restricted to this tile's own output
    // cells, which only this lane writes, after this read) and u^n of i+1
    load_prev(i, pvn);
    load_plane(i + 1, pn, plo, phi, ped);
    if (r >= z0 && r < z1) {
#pragma unroll
      for (int j = 0; j < kRows; ++j) {
        const int y = yb + j;
        if (y >= oy1) continue;  // wave-uniform
        const float4 cc = zc.v[j];
        const float4 ym = j == 0 ? hlo_c : zc.v[j - 1];
        const float4 yp = j == kRows - 1 ? hhi_c : zc.v[j + 1];
        const float4 zmv = zm.v[j], zpv = zp.v[j];
        const float left_n = dpp_from_left(cc.w);
        const float right_n = dpp_from_right(cc.x);
        const float xm0 = lane == 0 ? ed_c[j] : left_n;
        const float xp3 = lane == 63 ? ed_c[j] : right_n;
        float4 o;
        o.x = cell3(zmv.x, zpv.x, ym.x, yp.x, xm0, cc.y, cc.x, pv[j].x, r2);
        o.y = cell3(zmv.y, zpv.y, ym.y, yp.y, cc.x, cc.z, cc.y, pv[j].y, r2);
        o.z = cell3(zmv.z, zpv.z, ym.z, yp.z, cc.y, cc.w, cc.z, pv[j].z, r2);
        o.w = cell3(zmv.w, zpv.w, ym.w, yp.w, cc.z, xp3, cc.w, pv[j].w, r2);
        if (out.any) {
          // partial groups only at the chunk's x edges: merge with the
          // unchanged halo cells of this buffer, one 16-byte store
          float4 *p = reinterpret_cast<float4 *>(
              C.io_prev + static_cast<int64_t>(r - C.ip_z0) * C.ip_pz +
              static_cast<int64_t>(y - C.ip_y0) * C.ip_py + (xl - C.ip_x0));
          if (!(out.m0 && out.m1 && out.m2 && out.m3)) {
            const float4 q = *p;
            o.x = out.m0 ? o.x : q.x;
            o.y = out.m1 ? o.y : q.y;
            o.z = out.m2 ? o.z : q.z;
            o.w = out.m3 ? o.w : q.w;
          }
          *p = o;
        }
      }
    }
  }
}

bool fits_i32(int64_t v) { return v >= INT32_MIN && v <= INT32_MAX; }

int64_t wave_slots3d() {
  static int64_t cached = 0;
  if (cached > 0) return cached;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void *>(&wave3d_kernel<false>), kThreads, 0) !=
              hipSuccess ||
      per_cu < 1)
    return 1024;
  cached = static_cast<int64_t>(cus) * per_cu * kWavesPerBlock;
  return cached;
}

}  // namespace

int64_t wave3d_slots(int32_t T) { return T > 1 ? wave3d_tb_wave_slots(T) : wave_slots3d(); }

// The planes per tile the launcher would pick for a domain split into K
// plane chunks, at temporal depth T.
int32_t wave3d_plan_planes(int64_t nz, int64_t ny, int64_t nx, int32_t K, int32_t T) {
  if (T > 1) return wave3d_tb_plan_planes(nz, ny, nx, K, T);
  int64_t zmax = 0;
  for (int k = 0; k < K; ++k) zmax = std::max<int64_t>(zmax, (k + 1) * nz / K - k * nz / K);
  auto waves_of = [&](int32_t p) {
    int64_t w = 0;
    for (int k = 0; k < K; ++k) {
      const int64_t z = (k + 1) * nz / K - k * nz / K;
      w += ((z + p - 1) / p) * ((nx + 255) / 256) * ((ny + kRows - 1) / kRows);
    }
    return w;
  };
  return plan_tile_rows(wave_slots3d(), 1, 4, static_cast<int32_t>(std::max<int64_t>(zmax, 4)),
                        waves_of);
}

ccl_status launch_wave3d(int32_t depth, bool in_place, float r2, int32_t tile_planes,
                         const WaveChunkPlan *plans, int32_t nplans, hipStream_t stream) {
  if (depth > 1) {
    if (in_place) return fail(CCL_E_INVALID, "in-place update needs T == 1");
    return launch_wave3d_tb(depth, r2, tile_planes, plans, nplans, stream);
  }
  if (!in_place) return fail(CCL_E_INVALID, "the one-step 3D kernel updates in place");
  for (int first = 0; first < nplans; first += kMaxChunksPerLaunch) {
    const int n = std::min(kMaxChunksPerLaunch, nplans - first);
    W3Args a;
    memset(&a, 0, sizeof(a));
    a.nchunks = n;
    a.r2 = r2;
    if (tile_planes > 0) {
      a.tile_planes = tile_planes;
    } else {
      int64_t zmax = 0;
      for (int k = 0; k < n; ++k)
        zmax = std::max<int64_t>(zmax, plans[first + k].chunk.hi[0] - plans[first + k].chunk.lo[0]);
      auto waves_of = [&](int32_t p) {
        int64_t w = 0;
        for (int k = 0; k < n; ++k) {
          const Box &cb = plans[first + k].chunk;
          w += ((cb.hi[0] - cb.lo[0] + p - 1) / p) * ((cb.hi[2] - cb.lo[2] + 255) / 256) *
               ((cb.hi[1] - cb.lo[1] + kRows - 1) / kRows);
        }
        return w;
      };
      a.tile_planes = plan_tile_rows(wave_slots3d(), 1, 4,
                                     static_cast<int32_t>(std::max<int64_t>(zmax, 4)), waves_of);
    }
    int64_t tiles = 0;
    for (int k = 0; k < n; ++k) {
      const WaveChunkPlan &P = plans[first + k];
      W3Chunk &C = a.ch[k];
      C.in_cur = P.in_cur.base;
      C.io_prev = P.in_prev.base;
      for (int d = 0; d < 3; ++d)
        if (!fits_i32(P.in_cur.off[d]) || !fits_i32(P.in_prev.off[d]) ||
            !fits_i32(P.domain.lo[d] - 1024) || !fits_i32(P.domain.hi[d] + 1024))
          return fail(CCL_E_RANGE, "3D indices must fit in int32");
      C.ic_z0 = static_cast<int32_t>(P.in_cur.off[0]);
      C.ic_y0 = static_cast<int32_t>(P.in_cur.off[1]);
      C.ic_x0 = static_cast<int32_t>(P.in_cur.off[2]);
      C.ip_z0 = static_cast<int32_t>(P.in_prev.off[0]);
      C.ip_y0 = static_cast<int32_t>(P.in_prev.off[1]);
      C.ip_x0 = static_cast<int32_t>(P.in_prev.off[2]);
      C.ic_pz = P.in_cur.pitch[0];
      C.ic_py = P.in_cur.pitch[1];
      C.ip_pz = P.in_prev.pitch[0];
      C.ip_py = P.in_prev.pitch[1];
      C.lc_z0 = static_cast<int32_t>(P.load_cur.lo[0]);
      C.lc_z1 = static_cast<int32_t>(P.load_cur.hi[0]);
      C.lc_y0 = static_cast<int32_t>(P.load_cur.lo[1]);
      C.lc_y1 = static_cast<int32_t>(P.load_cur.hi[1]);
      C.lc_x0 = static_cast<int32_t>(P.load_cur.lo[2]);
      C.lc_x1 = static_cast<int32_t>(P.load_cur.hi[2]);
      C.cz0 = static_cast<int32_t>(P.chunk.lo[0]);
      C.cz1 = static_cast<int32_t>(P.chunk.hi[0]);
      C.cy0 = static_cast<int32_t>(P.chunk.lo[1]);
      C.cy1 = static_cast<int32_t>(P.chunk.hi[1]);
      C.cx0 = static_cast<int32_t>(P.chunk.lo[2]);
      C.cx1 = static_cast<int32_t>(P.chunk.hi[2]);
      // strip 0 starts at the chunk's first column aligned down to a
      // multiple of 4 relative to the u^n buffer, so every lane's group of
      // four columns is one 16-byte access; the output mask keeps the
      // columns left of the chunk unchanged
      const int64_t mis = (((P.chunk.lo[2] - P.in_cur.off[2]) % 4) + 4) % 4;
      const int64_t xs0 = P.chunk.lo[2] - mis;
      C.xs0 = static_cast<int32_t>(xs0);
      const int64_t nx = P.chunk.hi[2] - xs0;
      const int64_t ny = P.chunk.hi[1] - P.chunk.lo[1];
      const int64_t nz = P.chunk.hi[0] - P.chunk.lo[0];
      C.nstrips = static_cast<int32_t>((nx + 255) / 256);
      C.nrowblk = static_cast<int32_t>((ny + kRows - 1) / kRows);
      const int64_t segs = (nz + a.tile_planes - 1) / a.tile_planes;
      {
        // both buffers must hold the strips' groups at 16-byte boundaries
        const int64_t rp = xs0 - P.in_prev.off[2];
        if ((((rp % 4) + 4) % 4) != 0 || P.in_cur.pitch[0] % 4 != 0 ||
            P.in_cur.pitch[1] % 4 != 0 || P.in_prev.pitch[0] % 4 != 0 ||
            P.in_prev.pitch[1] % 4 != 0 ||
            (reinterpret_cast<uintptr_t>(P.in_cur.base) & 15u) != 0 ||
            (reinterpret_cast<uintptr_t>(P.in_prev.base) & 15u) != 0)
          return fail(CCL_E_INVALID,
                      "chunk %d: 3D buffers must be 16-byte aligned with pitches a multiple of 4 "
                      "and the same region column offset modulo 4",
                      first + k);
      }
      C.tile_begin = static_cast<int32_t>(tiles);
      tiles += segs * C.nstrips * C.nrowblk;
      if (tiles > INT32_MAX / 2) return fail(CCL_E_RANGE, "too many tiles");
    }
    a.total_tiles = static_cast<int32_t>(tiles);
    const int blocks = static_cast<int>((tiles + kWavesPerBlock - 1) / kWavesPerBlock);
    if (blocks == 0) continue;
    bool xin = true;  // every strip of every chunk fully interior in x
    for (int k = 0; k < n; ++k) {
      const W3Chunk &C = a.ch[k];
      xin = xin && C.xs0 == C.cx0 && (C.cx1 - C.cx0) % 256 == 0 && C.cx0 >= C.lc_x0 &&
            C.cx1 <= C.lc_x1;
    }
    ccl_status st;
    {
      TimedLaunch tl(CCL_KERNEL_STENCIL, stream);
      if (xin)
        hipLaunchKernelGGL(wave3d_kernel<true>, dim3(blocks), dim3(kThreads), 0, stream, a);
      else
        hipLaunchKernelGGL(wave3d_kernel<false>, dim3(blocks), dim3(kThreads), 0, stream, a);
    }
    st = hip_check(hipGetLastError(), "wave3d_kernel launch");
    if (st != CCL_OK) return st;
  }
  return CCL_OK;
}

}  // namespace ccl
