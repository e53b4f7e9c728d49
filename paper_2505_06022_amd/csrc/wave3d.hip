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
#include "prec.h"
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
  const void *in_cur;
  void *io_prev;  // u^{n-1} in, u^{n+1} out
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
  float r2f;   // r2 rounded to float (float arithmetic)
  double r2d;  // r2 as given (double arithmetic)
  W3Chunk ch[kMaxChunksPerLaunch];
};

template <class F>
__device__ __forceinline__ F r2_of(const W3Args &a);
template <>
__device__ __forceinline__ float r2_of<float>(const W3Args &a) { return a.r2f; }
template <>
__device__ __forceinline__ double r2_of<double>(const W3Args &a) { return a.r2d; }

template <class PR>
struct Plane {
  Vec<typename PR::F, PR::NV> v[kRows];
};

// Which of the lane's NV columns [xl, xl+NV) lie in [x0, x1).  Groups are
// aligned NV-tuples relative to the buffer and pitches are multiples of NV
// that cover the extent, so a group meeting [x0, x1) lies inside its row.
struct Cols {
  bool any;
  bool m[4];
};

template <int NV>
__device__ __forceinline__ Cols cols_of(int xl, int x0, int x1) {
  Cols c;
  c.any = false;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    c.m[i] = i < NV && xl + i >= x0 && xl + i < x1;
    c.any = c.any || c.m[i];
  }
  return c;
}

template <int NV>
__device__ __forceinline__ bool all_of(const Cols &c) {
  bool a = true;
#pragma unroll
  for (int i = 0; i < NV; ++i) a = a && c.m[i];
  return a;
}

template <class PR>
__device__ __forceinline__ Vec<typename PR::F, PR::NV> zero_v() {
  Vec<typename PR::F, PR::NV> z;
#pragma unroll
  for (int i = 0; i < PR::NV; ++i) z.v[i] = typename PR::F(0);
  return z;
}

template <class PR>
__device__ __forceinline__ Vec<typename PR::F, PR::NV> ld_group(
    const void *base, int64_t pz, int64_t py, int z0, int y0, int x0, int z, int y, int xl,
    int lz0, int lz1, int ly0, int ly1, const Cols &c) {
  using Raw = typename PR::Raw;
  Vec<typename PR::F, PR::NV> v = zero_v<PR>();
  if (z < lz0 || z >= lz1 || y < ly0 || y >= ly1) return v;  // wave-uniform
  Raw r;
#pragma unroll
  for (int i = 0; i < PR::NV; ++i) r[i] = typename PR::E(0);
  if (c.any)
    r = *reinterpret_cast<const Raw *>(static_cast<const typename PR::E *>(base) +
                                       static_cast<int64_t>(z - z0) * pz +
                                       static_cast<int64_t>(y - y0) * py + (xl - x0));
#pragma unroll
  for (int i = 0; i < PR::NV; ++i) v.v[i] = c.m[i] ? PR::widen(r[i]) : typename PR::F(0);
  return v;
}

__device__ __forceinline__ int xcd_block(int bid, int nblocks) {
  const int q = nblocks >> 3, r = nblocks & 7;
  const int xcd = bid & 7, idx = bid >> 3;
  return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + idx;
}

// XIN: the strip's 64*NV columns lie inside the loadable and the output
// column ranges (every strip of a domain whose width is a multiple of the
// strip width), so loads and stores need no per-element column masks.
template <class PR, bool XIN>
__global__ __launch_bounds__(kThreads) void wave3d_kernel(const W3Args a) {
  constexpr int NV = PR::NV;
  constexpr int SWD = 64 * NV;  // strip width
  using F = typename PR::F;
  using V = Vec<F, NV>;
  using E = typename PR::E;
  using Raw = typename PR::Raw;
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
  const int xs = C.xs0 + strip * SWD;
  const int xl = xs + NV * lane;
  const F r2 = r2_of<F>(a);

  Cols all;
  all.any = true;
#pragma unroll
  for (int i = 0; i < 4; ++i) all.m[i] = i < NV;
  // u^{n-1} is read (and written) only inside this tile's own output cells
  const int oy1 = min(C.cy1, yb + kRows);
  const Cols out = XIN ? all : cols_of<NV>(xl, C.cx0, C.cx1);
  const Cols lc = XIN ? all : cols_of<NV>(xl, C.lc_x0, C.lc_x1);
  const int edge_x = lane == 0 ? xs - 1 : xs + SWD;
  const bool edge_lane = lane == 0 || lane == 63;

  Plane<PR> zm, zc, zp;  // ring: planes r-1, r, r+1 (r = centre)
  V hlo_c, hhi_c, hlo_n, hhi_n;  // halo rows of the centre / newest plane
  F ed_c[kRows], ed_n[kRows];    // outer columns of the centre / newest plane
#pragma unroll
  for (int j = 0; j < kRows; ++j) {
    zm.v[j] = zc.v[j] = zp.v[j] = zero_v<PR>();
    ed_c[j] = ed_n[j] = F(0);
  }
  hlo_c = hhi_c = hlo_n = hhi_n = zero_v<PR>();

  auto load_plane = [&](int z, Plane<PR> &pl, V &hlo, V &hhi, F *ed) {
#pragma unroll
    for (int j = 0; j < kRows; ++j)
      pl.v[j] = ld_group<PR>(C.in_cur, C.ic_pz, C.ic_py, C.ic_z0, C.ic_y0, C.ic_x0, z, yb + j, xl,
                             C.lc_z0, C.lc_z1, C.lc_y0, C.lc_y1, lc);
    hlo = ld_group<PR>(C.in_cur, C.ic_pz, C.ic_py, C.ic_z0, C.ic_y0, C.ic_x0, z, yb - 1, xl,
                       C.lc_z0, C.lc_z1, C.lc_y0, C.lc_y1, lc);
    hhi = ld_group<PR>(C.in_cur, C.ic_pz, C.ic_py, C.ic_z0, C.ic_y0, C.ic_x0, z, yb + kRows, xl,
                       C.lc_z0, C.lc_z1, C.lc_y0, C.lc_y1, lc);
    const bool zin = z >= C.lc_z0 && z < C.lc_z1;
    const bool xin = edge_x >= C.lc_x0 && edge_x < C.lc_x1;
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      const int y = yb + j;
      F e = F(0);
      if (edge_lane && zin && xin && y >= C.lc_y0 && y < C.lc_y1)
        e = PR::widen(static_cast<const E *>(C.in_cur)[static_cast<int64_t>(z - C.ic_z0) * C.ic_pz +
                                                       static_cast<int64_t>(y - C.ic_y0) * C.ic_py +
                                                       (edge_x - C.ic_x0)]);
      ed[j] = e;
    }
  };

  auto load_prev = [&](int z, V *pv) {
#pragma unroll
    for (int j = 0; j < kRows; ++j)
      pv[j] = ld_group<PR>(C.io_prev, C.ip_pz, C.ip_py, C.ip_z0, C.ip_y0, C.ip_x0, z, yb + j, xl,
                           z0, z1, yb, oy1, out);
  };

  const int i0 = z0 - 1;
  // prime: plane z0-1 becomes the centre plane after the first shift
  load_plane(i0, zp, hlo_n, hhi_n, ed_n);
  Plane<PR> pn;
  V plo, phi;
  F ped[kRows];
  load_plane(i0 + 1, pn, plo, phi, ped);
  V pv[kRows], pvn[kRows];
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
        const V cc = zc.v[j];
        const V ym = j == 0 ? hlo_c : zc.v[j - 1];
        const V yp = j == kRows - 1 ? hhi_c : zc.v[j + 1];
        const V zmv = zm.v[j], zpv = zp.v[j];
        const F left_n = dpp_move<0x138>(cc.v[NV - 1]);   // wave_shr:1
        const F right_n = dpp_move<0x130>(cc.v[0]);       // wave_shl:1
        const F xm0 = lane == 0 ? ed_c[j] : left_n;
        const F xpl = lane == 63 ? ed_c[j] : right_n;
        Raw o;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          const F xm = q == 0 ? xm0 : cc.v[q > 0 ? q - 1 : 0];
          const F xp = q == NV - 1 ? xpl : cc.v[q < NV - 1 ? q + 1 : 0];
          o[q] = PR::narrow(cell3(zmv.v[q], zpv.v[q], ym.v[q], yp.v[q], xm, xp, cc.v[q],
                                  pv[j].v[q], r2));
        }
        if (out.any) {
          // partial groups only at the chunk's x edges: merge with the
          // unchanged halo cells of this buffer, one vector store
          Raw *p = reinterpret_cast<Raw *>(
              static_cast<E *>(C.io_prev) + static_cast<int64_t>(r - C.ip_z0) * C.ip_pz +
              static_cast<int64_t>(y - C.ip_y0) * C.ip_py + (xl - C.ip_x0));
          if (!all_of<NV>(out)) {
            const Raw q = *p;
#pragma unroll
            for (int e = 0; e < NV; ++e) o[e] = out.m[e] ? o[e] : q[e];
          }
          *p = o;
        }
      }
    }
  }
}

template <class PR>
const void *kernel_of(bool xin) {
  return xin ? reinterpret_cast<const void *>(&wave3d_kernel<PR, true>)
             : reinterpret_cast<const void *>(&wave3d_kernel<PR, false>);
}

const void *kernel_for(int32_t dtype, bool xin) {
  switch (dtype) {
    case CCL_DTYPE_F64: return kernel_of<P64>(xin);
    case CCL_DTYPE_BF16: return kernel_of<PB16>(xin);
    case CCL_DTYPE_F16: return kernel_of<PH16>(xin);
    default: return kernel_of<P32>(xin);
  }
}

bool fits_i32(int64_t v) { return v >= INT32_MIN && v <= INT32_MAX; }

int64_t wave_slots3d(int32_t dtype = CCL_DTYPE_F32) {
  static int64_t cached[4] = {};
  if (dtype < 0 || dtype > 3) dtype = CCL_DTYPE_F32;
  if (cached[dtype] > 0) return cached[dtype];
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel_for(dtype, false), kThreads,
                                                    0) != hipSuccess ||
      per_cu < 1)
    return 1024;
  cached[dtype] = static_cast<int64_t>(cus) * per_cu * kWavesPerBlock;
  return cached[dtype];
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

ccl_status launch_wave3d(int32_t dtype, int32_t depth, bool in_place, double r2,
                         int32_t tile_planes, const WaveChunkPlan *plans, int32_t nplans,
                         hipStream_t stream) {
  if (depth > 1) {
    if (in_place) return fail(CCL_E_INVALID, "in-place update needs T == 1");
    return launch_wave3d_tb(dtype, depth, r2, tile_planes, plans, nplans, stream);
  }
  const int NV = dtype_group(dtype);
  const int esize = dtype_bytes(dtype);
  if (esize == 0) return fail(CCL_E_INVALID, "unknown dtype %d", dtype);
  const int SWD = 64 * NV;
  const uintptr_t amask = static_cast<uintptr_t>(NV * esize - 1);
  if (!in_place) return fail(CCL_E_INVALID, "the one-step 3D kernel updates in place");
  for (int first = 0; first < nplans; first += kMaxChunksPerLaunch) {
    const int n = std::min(kMaxChunksPerLaunch, nplans - first);
    W3Args a;
    memset(&a, 0, sizeof(a));
    a.nchunks = n;
    a.r2f = static_cast<float>(r2);
    a.r2d = r2;
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
          w += ((cb.hi[0] - cb.lo[0] + p - 1) / p) * ((cb.hi[2] - cb.lo[2] + SWD - 1) / SWD) *
               ((cb.hi[1] - cb.lo[1] + kRows - 1) / kRows);
        }
        return w;
      };
      a.tile_planes = plan_tile_rows(wave_slots3d(dtype), 1, 4,
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
      // multiple of NV relative to the u^n buffer, so every lane's group of
      // NV columns is one aligned vector access; the output mask keeps the
      // columns left of the chunk unchanged
      const int64_t mis = (((P.chunk.lo[2] - P.in_cur.off[2]) % NV) + NV) % NV;
      const int64_t xs0 = P.chunk.lo[2] - mis;
      C.xs0 = static_cast<int32_t>(xs0);
      const int64_t nx = P.chunk.hi[2] - xs0;
      const int64_t ny = P.chunk.hi[1] - P.chunk.lo[1];
      const int64_t nz = P.chunk.hi[0] - P.chunk.lo[0];
      C.nstrips = static_cast<int32_t>((nx + SWD - 1) / SWD);
      C.nrowblk = static_cast<int32_t>((ny + kRows - 1) / kRows);
      const int64_t segs = (nz + a.tile_planes - 1) / a.tile_planes;
      {
        // both buffers must hold the strips' groups at aligned boundaries
        const int64_t rp = xs0 - P.in_prev.off[2];
        if ((((rp % NV) + NV) % NV) != 0 || P.in_cur.pitch[0] % NV != 0 ||
            P.in_cur.pitch[1] % NV != 0 || P.in_prev.pitch[0] % NV != 0 ||
            P.in_prev.pitch[1] % NV != 0 ||
            (reinterpret_cast<uintptr_t>(P.in_cur.base) & amask) != 0 ||
            (reinterpret_cast<uintptr_t>(P.in_prev.base) & amask) != 0)
          return fail(CCL_E_INVALID,
                      "chunk %d: 3D buffers must be %d-byte aligned with pitches a multiple of "
                      "%d and the same region column offset modulo %d",
                      first + k, NV * esize, NV, NV);
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
      xin = xin && C.xs0 == C.cx0 && (C.cx1 - C.cx0) % SWD == 0 && C.cx0 >= C.lc_x0 &&
            C.cx1 <= C.lc_x1;
    }
    ccl_status st;
    {
      TimedLaunch tl(CCL_KERNEL_STENCIL, stream);
      void *args[] = {&a};
      st = hip_check(hipLaunchKernel(kernel_for(dtype, xin), dim3(blocks), dim3(kThreads), args, 0,
                                     stream),
                     "wave3d_kernel launch");
      if (st != CCL_OK) return st;
    }
    st = hip_check(hipGetLastError(), "wave3d_kernel launch");
    if (st != CCL_OK) return st;
  }
  return CCL_OK;
}

}  // namespace ccl
