// 3D seven-point leapfrog stencil, T = 2..8 steps per pass over HBM.
//
// Work unit: one block of 1024 threads (16 waves, the most a CU holds at
// up to 128 VGPRs per lane) owns a patch of 16*NV columns by 64*P rows and
// streams along z through a segment of planes.  Thread (ly, lx) holds NV
// consecutive columns (one vector group: four floats, two doubles or four
// 16-bit values; see prec.h) of P consecutive rows (P = 1); the 16 threads
// of a patch row are one DPP row, so x-neighbours come from DPP row shifts.
// A taller patch re-computes less of its overlap with the neighbouring
// patches (at T = 6 a 64 x 64 patch stores 48 x 52 cells, a 64 x 32 patch
// 48 x 20).  For every level l < T the thread keeps the last three planes
// of u^{n+l} over its cells in registers (a rotating three-slot ring), so
// z-neighbours are register reads.  y-neighbours inside a thread's P rows
// are its own registers; the first and last of its rows take their outer
// neighbour from the adjacent thread row, published in LDS once per plane
// (one 16-byte word per thread and level when P = 1, two when P > 1; one
// barrier per plane).  One row per thread in 16 waves, rather than two rows
// in 8 waves, halves the registers per lane (111 against 204 at T = 6) and
// doubles the waves each SIMD can switch between while others wait on
// memory or the barrier: 11-13% faster at T = 6..8 on 768^3.
//
// At iteration i the block loads plane i of u^n (level 0) and, level by
// level, computes plane i-l of u^{n+l}; level T gives u^{n+T} at plane i-T,
// stored with u^{n+T-1} of the same plane.  A level-l value is valid only
// where its whole dependency cone was loaded, so patches overlap their
// neighbours by A = NV*ceil(T/NV) columns and T rows on each side and
// segments re-read T planes above and below; only the valid interior is
// stored.  Every cell is produced by the same expression as the one-step
// kernel, so results are bitwise independent of tiling (and of T where
// storage and arithmetic types agree).
#include <algorithm>
#include <cstring>
#include <type_traits>

#include "ccl_internal.h"
#include "prec.h"
#include "wave2d_tile.h"
#include "wave3d_cell.h"

namespace ccl {
namespace {

// Block shape: kThreads threads in rows of kLX; a patch row is kLX groups
// of NV columns and the patch has kThreads / kLX thread rows.
#ifndef CCL_W3T_THREADS
#define CCL_W3T_THREADS 1024
#endif
#ifndef CCL_W3T_LX
#define CCL_W3T_LX 16
#endif
constexpr int kThreads = CCL_W3T_THREADS;
constexpr int kLX = CCL_W3T_LX;
constexpr int kLY = kThreads / kLX;
static_assert(kLX == 16 || kLX == 32 || kLX == 64, "a patch row is 16, 32 or 64 lanes");
static_assert(kThreads % 64 == 0 && kThreads % kLX == 0, "whole waves and thread rows");
static_assert((kThreads & (kThreads - 1)) == 0, "row neighbours wrap with a power-of-two mask");
constexpr int kMaxChunksPerLaunch = 8;

// Rows per thread, planes loaded ahead, overlap, output extent and LDS
// buffering for depth T.
#ifndef CCL_W3T_ROWS
#define CCL_W3T_ROWS 1
#endif
__host__ __device__ constexpr int tb_rows(int) { return CCL_W3T_ROWS; }
#ifndef CCL_W3T_PF
__host__ __device__ constexpr int tb_prefetch(int) { return 1; }
#else
__host__ __device__ constexpr int tb_prefetch(int) { return CCL_W3T_PF; }
#endif
__host__ __device__ constexpr int tb_patch_cols(int NV) { return NV * kLX; }
__host__ __device__ constexpr int tb_overlap(int T, int NV = 4) { return NV * ((T + NV - 1) / NV); }
__host__ __device__ constexpr int tb_out_cols(int T, int NV = 4) {
  return tb_patch_cols(NV) - 2 * tb_overlap(T, NV);
}
__host__ __device__ constexpr int tb_out_rows(int T) { return kLY * tb_rows(T) - 2 * T; }
static_assert(tb_out_cols(CCL_MAX_DEPTH, 2) > 0 && tb_out_rows(CCL_MAX_DEPTH) > 0,
              "every depth leaves an interior to store");
// LDS words each thread publishes per level and plane: its first and its
// last row (one, when it holds a single row).
__host__ __device__ constexpr int tb_words(int T) { return tb_rows(T) > 1 ? 2 : 1; }
#ifndef CCL_W3T_NB
// Two buffers (one barrier per plane) where they fit in the 160 KiB of LDS,
// else one (a second barrier before the words are overwritten).
__host__ __device__ constexpr int tb_lds_buffers(int T) {
  return 2 * T * tb_words(T) * kThreads * 16 <= 160 * 1024 ? 2 : 1;
}
#else
__host__ __device__ constexpr int tb_lds_buffers(int) { return CCL_W3T_NB; }
#endif

struct Field3 {  // a chunk buffer: global index of its first element, strides
  int32_t z0, y0, x0;
  int32_t pz, py;
};

struct W3TChunk {
  const void *in_prev;
  const void *in_cur;
  void *out_prev;
  void *out_cur;
  Field3 ip, ic, op, oc;
  int32_t lp[6];  // loadable box of in_prev: z0, z1, y0, y1, x0, x1
  int32_t lc[6];  // loadable box of in_cur
  int32_t cz0, cz1, cy0, cy1, cx0, cx1;  // chunk (output) box
  int32_t xs0;                           // origin column of strip 0's patches
  int32_t nstrips, nrowblk;
  int32_t tile_begin;
};

struct W3TArgs {
  int32_t nchunks;
  int32_t total_tiles;
  int32_t tile_planes;
  float r2f;   // r2 rounded to float (float arithmetic)
  double r2d;  // r2 as given (double arithmetic)
  int32_t gz0, gz1, gy0, gy1, gx0, gx1;  // domain: zero outside
  W3TChunk ch[kMaxChunksPerLaunch];
};

template <class F>
__device__ __forceinline__ F r2_of(const W3TArgs &a);
template <>
__device__ __forceinline__ float r2_of<float>(const W3TArgs &a) { return a.r2f; }
template <>
__device__ __forceinline__ double r2_of<double>(const W3TArgs &a) { return a.r2d; }

// x-neighbours across the lanes of a patch row.  16-lane rows are DPP rows
// (row_shr:1 / row_shl:1); wider rows use the wave shifts (wave_shr:1 /
// wave_shl:1), where the first lane of the second row of a wave receives
// the last lane of the first: a patch-edge cell, never valid, so harmless.
template <class F>
__device__ __forceinline__ F row_from_left(F v) {
  return dpp_move<kLX == 16 ? 0x111 : 0x138>(v);
}
template <class F>
__device__ __forceinline__ F row_from_right(F v) {
  return dpp_move<kLX == 16 ? 0x101 : 0x130>(v);
}

// One buffer as the streaming loop sees it: its base, the plane index of
// its origin and the plane stride (block-uniform), and per thread the
// element offset, within a plane, of each of the thread's rows (32 bits:
// strides are checked to fit in int32 on the host).  A row that the
// buffer does not hold has an offset that is never used.
template <class E, int P>
struct Rows {
  const E *base;
  int32_t z0;
  int32_t pz;
  uint32_t off[P];
};

template <class E, int P>
__device__ __forceinline__ Rows<E, P> rows_of(const void *base, const Field3 &f, int yl, int xl) {
  Rows<E, P> r;
  r.base = static_cast<const E *>(base);
  r.z0 = f.z0;
  r.pz = f.pz;
#pragma unroll
  for (int j = 0; j < P; ++j)
    r.off[j] = static_cast<uint32_t>((yl + j - f.y0) * f.py + (xl - f.x0));
  return r;
}

template <class E, int P>
__device__ __forceinline__ const E *plane_of(const Rows<E, P> &b, int z) {
  return b.base + static_cast<int64_t>(z - b.z0) * b.pz;
}

// The thread's P rows of plane z, widened: zero outside the loadable box
// (planes [lz0, lz1), rows where ok[j], columns in cx).  STREAM marks data
// read once (u^{n-1}).
template <class PR, bool STREAM, int P>
__device__ __forceinline__ void load_rows(Vec<typename PR::F, PR::NV> (&v)[P],
                                          const Rows<typename PR::E, P> &b, int z, int lz0,
                                          int lz1, const bool (&ok)[P], const w2::Cols &cx) {
  using Raw = typename PR::Raw;
  using F = typename PR::F;
  const bool zin = z >= lz0 && z < lz1;  // block-uniform
  const typename PR::E *plane = plane_of(b, z);
#pragma unroll
  for (int j = 0; j < P; ++j) {
    Raw q;
#pragma unroll
    for (int i = 0; i < PR::NV; ++i) q[i] = typename PR::E(0);
    if (zin && ok[j] && cx.any) {
      const Raw *p = reinterpret_cast<const Raw *>(plane + b.off[j]);
      q = STREAM ? __builtin_nontemporal_load(p) : *p;
    }
#pragma unroll
    for (int i = 0; i < PR::NV; ++i) v[j].v[i] = cx.m[i] ? PR::widen(q[i]) : F(0);
  }
}

// Stores a group where the output mask allows, narrowed to the storage
// type.  Partial groups occur only at a chunk's x edges; their other
// columns are halo cells of this chunk's own output buffer that nothing
// writes during the launch, so they are read and written back unchanged
// (one vector store).
template <class PR>
__device__ __forceinline__ void store_group(typename PR::E *p_, const w2::Cols &c,
                                            const Vec<typename PR::F, PR::NV> &v) {
  using Raw = typename PR::Raw;
  Raw *p = reinterpret_cast<Raw *>(p_);
  Raw w;
#pragma unroll
  for (int i = 0; i < PR::NV; ++i) w[i] = PR::narrow(v.v[i]);
  if (!w2::all_of<PR::NV>(c)) {
    const Raw o = *p;
#pragma unroll
    for (int i = 0; i < PR::NV; ++i) w[i] = c.m[i] ? w[i] : o[i];
  }
  __builtin_nontemporal_store(w, p);
}

// What the streaming loop of one block needs, gathered once (in registers,
// so nothing is reloaded from the kernel arguments after a store).
template <class PR, int P>
struct Patch {
  using E = typename PR::E;
  Rows<E, P> ic, ip, oc, op;
  int32_t lc_z0, lc_z1, lp_z0, lp_z1;  // loadable planes of u^n, u^{n-1}
  int32_t gz0, gz1;                     // domain planes
  int32_t zo0, zo1;                     // output planes of this segment
  bool ok_c[P], ok_p[P], out_row[P], dom_row[P];
  w2::Cols lcx, lpx, dom, out;
  bool xy_in;                           // patch inside the domain in x and y
};

// xch: the block's LDS words, [buffer][level][first row / last row][thread]
// (one row, and one word, when a thread holds a single row); each word is
// one thread's group of NV arithmetic values (16 bytes).
template <class PR, int T>
__device__ __forceinline__ void stream_patch(const Patch<PR, tb_rows(T)> &S, typename PR::F r2,
                                             int tid,
                                             Vec<typename PR::F, PR::NV> (*xch)[T][tb_words(T)][kThreads]) {
  constexpr int P = tb_rows(T);
  constexpr int NB = tb_lds_buffers(T);
  constexpr int PF = tb_prefetch(T);
  constexpr int NV = PR::NV;
  using F = typename PR::F;
  using V = Vec<F, NV>;
  static_assert(PF == 1 || PF == 3, "prefetch depth is 1 or 3 planes");

  V ring[T][3][P];  // level l: planes i-l-2, i-l-1, i-l in rotating slots
#pragma unroll
  for (int l = 0; l < T; ++l)
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
      for (int j = 0; j < P; ++j)
#pragma unroll
        for (int q = 0; q < NV; ++q) ring[l][s][j].v[q] = F(0);

  const int i0 = S.zo0 - T;
  const int n_iter = (S.zo1 - S.zo0) + 2 * T;
  // planes loaded ahead: u^n of planes i..i+PF-1 and u^{n-1} of the plane
  // before each; with PF = 3 plane i sits in slot i - i0 mod 3, the
  // iteration's phase, so the slots rotate without moves
  V qs[PF][P], ps[PF][P];
#pragma unroll
  for (int f = 0; f < PF; ++f) {
    load_rows<PR, false>(qs[f], S.ic, i0 + f, S.lc_z0, S.lc_z1, S.ok_c, S.lcx);
    load_rows<PR, true>(ps[f], S.ip, i0 + f - 1, S.lp_z0, S.lp_z1, S.ok_p, S.lpx);
  }

  // One iteration; PH = iteration count mod 3 names the ring slots: before
  // it the newest plane of every level sits in slot (PH+2)%3, after it in
  // slot PH, with the middle in (PH+2)%3 and the oldest in (PH+1)%3.
  auto iteration = [&](auto ph, auto warm, int i) {
    constexpr int PH = decltype(ph)::value;
    constexpr bool WARM = decltype(warm)::value;
    constexpr int NEW = PH, MID = (PH + 2) % 3, OLD = (PH + 1) % 3;
    const int b = NB == 2 ? (i & 1) : 0;
    if (NB == 1) __syncthreads();  // every thread has read the last plane's words
#pragma unroll
    for (int l = 0; l < T; ++l) {
      xch[b][l][0][tid] = ring[l][MID][0];  // MID is still the newest here
      if constexpr (P > 1) xch[b][l][P > 1 ? 1 : 0][tid] = ring[l][MID][P - 1];
    }
    __syncthreads();

    // level 0: plane i of u^n arrives; u^{n-1} of plane i-1 for level 1
    constexpr int QS = PF == 3 ? PH : 0;
#pragma unroll
    for (int j = 0; j < P; ++j) ring[0][NEW][j] = qs[QS][j];
    V pc[P];
#pragma unroll
    for (int j = 0; j < P; ++j) pc[j] = ps[QS][j];
    load_rows<PR, false>(qs[QS], S.ic, i + PF, S.lc_z0, S.lc_z1, S.ok_c, S.lcx);
    load_rows<PR, true>(ps[QS], S.ip, i + PF - 1, S.lp_z0, S.lp_z1, S.ok_p, S.lpx);

#pragma unroll
    for (int t = 1; t <= T; ++t) {
      // warm-up: level t of this iteration's plane feeds a stored output
      // only from the 2t-th iteration on (block-uniform; levels above a
      // skipped one are skipped too)
      if (WARM && i - i0 < 2 * t) break;
      const int r = i - t;  // plane of u^{n+t} computed now
      const bool z_in = r >= S.gz0 && r < S.gz1;  // block-uniform
      // outer y-neighbours of this thread's rows in plane r of u^{n+t-1}
      // (the top thread row reads the bottom one's words: patch-edge cells
      // are never valid, so any value there is harmless)
      const V up = xch[b][t - 1][P > 1 ? 1 : 0][(tid - kLX) & (kThreads - 1)];
      const V dn = xch[b][t - 1][0][(tid + kLX) & (kThreads - 1)];
      V o[P];
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const V cc = ring[t - 1][MID][j];
        const V zm = ring[t - 1][OLD][j];
        const V zp = ring[t - 1][NEW][j];
        const V ym = j == 0 ? up : ring[t - 1][MID][j > 0 ? j - 1 : 0];
        const V yp = j == P - 1 ? dn : ring[t - 1][MID][j < P - 1 ? j + 1 : 0];
        const V pv = t == 1 ? pc[j] : ring[t >= 2 ? t - 2 : 0][OLD][j];
        const F xm0 = row_from_left(cc.v[NV - 1]);
        const F xpl = row_from_right(cc.v[0]);
        V v;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          const F xm = q == 0 ? xm0 : cc.v[q > 0 ? q - 1 : 0];
          const F xp = q == NV - 1 ? xpl : cc.v[q < NV - 1 ? q + 1 : 0];
          v.v[q] = cell3(zm.v[q], zp.v[q], ym.v[q], yp.v[q], xm, xp, cc.v[q], pv.v[q], r2);
        }
        if (!(S.xy_in && z_in)) {
          const bool in = z_in && S.dom_row[j];
#pragma unroll
          for (int q = 0; q < NV; ++q) v.v[q] = (in && S.dom.m[q]) ? v.v[q] : F(0);
        }
        o[j] = v;
      }
      if (t < T) {
#pragma unroll
        for (int j = 0; j < P; ++j) ring[t < T ? t : 0][NEW][j] = o[j];
      } else if (r >= S.zo0 && r < S.zo1 && S.out.any) {
        typename PR::E *pcur = const_cast<typename PR::E *>(plane_of(S.oc, r));
        typename PR::E *pprev = const_cast<typename PR::E *>(plane_of(S.op, r));
#pragma unroll
        for (int j = 0; j < P; ++j) {
          if (!S.out_row[j]) continue;
          store_group<PR>(pcur + S.oc.off[j], S.out, o[j]);
          store_group<PR>(pprev + S.op.off[j], S.out, ring[T - 1][MID][j]);
        }
      }
    }
  };

  // The first 2T iterations (in whole turns of the ring) skip the levels
  // whose planes no stored output needs yet: level t at iteration i0 + m
  // lies on plane i0 + m - t, and the outputs' dependency cone needs level
  // t only from plane i0 + t on.  What a computed level reads was computed
  // (levels t-1 and t-2 from iteration m-2 >= 2(t-1) on), so stored values
  // are unchanged; T(T+1) of the segment's T * n_iter level-planes are
  // skipped (768^3 at T = 7: 2.6% faster).  At T = 8 the second copy of the
  // loop pushes the kernel past 128 VGPRs into spills (15% slower), so the
  // deepest kernel keeps the single loop.
  using warm = std::true_type;
  using steady = std::false_type;
  int n = 0;
  if constexpr (T < CCL_MAX_DEPTH) {
    const int n_warm = min(n_iter, 3 * ((2 * T + 2) / 3));
    for (; n < n_warm; n += 3) {
      iteration(std::integral_constant<int, 0>(), warm(), i0 + n);
      if (n + 1 < n_iter) iteration(std::integral_constant<int, 1>(), warm(), i0 + n + 1);
      if (n + 2 < n_iter) iteration(std::integral_constant<int, 2>(), warm(), i0 + n + 2);
    }
  }
  for (; n < n_iter; n += 3) {
    iteration(std::integral_constant<int, 0>(), steady(), i0 + n);
    if (n + 1 < n_iter) iteration(std::integral_constant<int, 1>(), steady(), i0 + n + 1);
    if (n + 2 < n_iter) iteration(std::integral_constant<int, 2>(), steady(), i0 + n + 2);
  }
}

template <class PR, int T>
__global__ __launch_bounds__(kThreads) void wave3d_tb_kernel(const W3TArgs a) {
  constexpr int NV = PR::NV;
  constexpr int P = tb_rows(T);
  constexpr int A = tb_overlap(T, NV);
  constexpr int OW = tb_out_cols(T, NV);
  constexpr int OH = tb_out_rows(T);
  using E = typename PR::E;
  using F = typename PR::F;

  const int blk = w2::xcd_block(blockIdx.x, gridDim.x);
  if (blk >= a.total_tiles) return;  // the whole block leaves together
  int c = 0;
  while (c + 1 < a.nchunks && blk >= a.ch[c + 1].tile_begin) ++c;
  const W3TChunk &C = a.ch[c];

  // tile order: strip fastest, then row block, then z segment
  int local = blk - C.tile_begin;
  const int per_seg = C.nstrips * C.nrowblk;
  const int seg = local / per_seg;
  local -= seg * per_seg;
  const int rb = local / C.nstrips;
  const int strip = local - rb * C.nstrips;

  const int tid = threadIdx.x;
  const int lx = tid % kLX, ly = tid / kLX;
  const int px = C.xs0 + strip * OW;  // patch origin
  const int py = C.cy0 - T + rb * OH;
  const int xl = px + NV * lx;
  const int yl = py + ly * P;
  const int oy0 = max(C.cy0, py + T), oy1 = min(C.cy1, py + T + OH);

  Patch<PR, P> S;
  S.ic = rows_of<E, P>(C.in_cur, C.ic, yl, xl);
  S.ip = rows_of<E, P>(C.in_prev, C.ip, yl, xl);
  S.oc = rows_of<E, P>(C.out_cur, C.oc, yl, xl);
  S.op = rows_of<E, P>(C.out_prev, C.op, yl, xl);
  S.lc_z0 = C.lc[0];
  S.lc_z1 = C.lc[1];
  S.lp_z0 = C.lp[0];
  S.lp_z1 = C.lp[1];
  S.gz0 = a.gz0;
  S.gz1 = a.gz1;
  S.zo0 = C.cz0 + seg * a.tile_planes;
  S.zo1 = min(C.cz1, S.zo0 + a.tile_planes);
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int y = yl + j;
    S.ok_c[j] = y >= C.lc[2] && y < C.lc[3];
    S.ok_p[j] = y >= C.lp[2] && y < C.lp[3];
    S.out_row[j] = y >= oy0 && y < oy1;
    S.dom_row[j] = y >= a.gy0 && y < a.gy1;
  }
  S.lcx = w2::cols_of<NV>(xl, C.lc[4], C.lc[5]);
  S.lpx = w2::cols_of<NV>(xl, C.lp[4], C.lp[5]);
  S.dom = w2::cols_of<NV>(xl, a.gx0, a.gx1);
  S.out = w2::cols_of<NV>(xl, max(C.cx0, px + A), min(C.cx1, px + A + OW));
  S.xy_in = px >= a.gx0 && px + tb_patch_cols(NV) <= a.gx1 && py >= a.gy0 &&
            py + kLY * P <= a.gy1;
  __shared__ Vec<F, NV> xch[tb_lds_buffers(T)][T][tb_words(T)][kThreads];
  stream_patch<PR, T>(S, r2_of<F>(a), tid, xch);
}

template <class PR, int T>
const void *kernel_of() {
  return reinterpret_cast<const void *>(&wave3d_tb_kernel<PR, T>);
}

template <class PR>
const void *kernel_depth(int T) {
  switch (T) {
    case 2: return kernel_of<PR, 2>();
    case 3: return kernel_of<PR, 3>();
    case 4: return kernel_of<PR, 4>();
    case 5: return kernel_of<PR, 5>();
    case 6: return kernel_of<PR, 6>();
    case 7: return kernel_of<PR, 7>();
    case 8: return kernel_of<PR, 8>();
    default: return nullptr;
  }
}

const void *kernel_for(int32_t dtype, int T) {
  switch (dtype) {
    case CCL_DTYPE_F32: return kernel_depth<P32>(T);
    case CCL_DTYPE_F64: return kernel_depth<P64>(T);
    case CCL_DTYPE_BF16: return kernel_depth<PB16>(T);
    case CCL_DTYPE_F16: return kernel_depth<PH16>(T);
    default: return nullptr;
  }
}

// Concurrently resident blocks of the depth-T kernel on the device (cached).
int64_t block_slots(int T, int32_t dtype = CCL_DTYPE_F32) {
  static int64_t cache[4][CCL_MAX_DEPTH + 1] = {};
  if (T < 2 || T > CCL_MAX_DEPTH || dtype < 0 || dtype > 3) return 256;
  if (cache[dtype][T] > 0) return cache[dtype][T];
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel_for(dtype, T), kThreads, 0) !=
          hipSuccess ||
      per_cu < 1)
    return 256;
  cache[dtype][T] = static_cast<int64_t>(cus) * per_cu;
  return cache[dtype][T];
}

int64_t tiles_of(int64_t nz, int64_t ny, int64_t nx, int T, int32_t planes, int NV = 4) {
  return ((nz + planes - 1) / planes) * ((ny + tb_out_rows(T) - 1) / tb_out_rows(T)) *
         ((nx + tb_out_cols(T, NV) - 1) / tb_out_cols(T, NV));
}

bool fits_i32(int64_t v) { return v >= INT32_MIN && v <= INT32_MAX; }

ccl_status field3_of(const WaveField &w, Field3 *f) {
  for (int d = 0; d < 3; ++d)
    if (!fits_i32(w.off[d])) return fail(CCL_E_RANGE, "3D buffer origins must fit in int32");
  if (!fits_i32(w.pitch[0]) || !fits_i32(w.pitch[1]))
    return fail(CCL_E_RANGE, "3D buffer strides must fit in int32");
  f->z0 = static_cast<int32_t>(w.off[0]);
  f->y0 = static_cast<int32_t>(w.off[1]);
  f->x0 = static_cast<int32_t>(w.off[2]);
  f->pz = static_cast<int32_t>(w.pitch[0]);
  f->py = static_cast<int32_t>(w.pitch[1]);
  return CCL_OK;
}

void box6(const Box &b, int32_t *o) {
  for (int d = 0; d < 3; ++d) {
    o[2 * d] = static_cast<int32_t>(b.lo[d]);
    o[2 * d + 1] = static_cast<int32_t>(b.hi[d]);
  }
}

ccl_status launch_k(const void *fn, const W3TArgs &a, int blocks, hipStream_t s) {
  if (!fn) return fail(CCL_E_INVALID, "no 3D blocked kernel for this dtype and depth");
  TimedLaunch tl(CCL_KERNEL_STENCIL, s);
  void *args[] = {const_cast<W3TArgs *>(&a)};
  return hip_check(hipLaunchKernel(fn, dim3(blocks), dim3(kThreads), args, 0, s),
                   "wave3d_tb_kernel launch");
}

}  // namespace

int64_t wave3d_tb_wave_slots(int32_t T) { return block_slots(T) * (kThreads / 64); }

void wave3d_tb_geometry(int32_t T, int32_t *out_cols, int32_t *out_rows, int32_t *waves) {
  *out_cols = tb_out_cols(T);
  *out_rows = tb_out_rows(T);
  *waves = kThreads / 64;
}

// Planes per z segment the depth-T kernel would pick for a domain split
// into K plane chunks (every block streams planes + 2T planes).
int32_t wave3d_tb_plan_planes(int64_t nz, int64_t ny, int64_t nx, int32_t K, int32_t T) {
  int64_t zmax = 0;
  for (int k = 0; k < K; ++k) zmax = std::max<int64_t>(zmax, (k + 1) * nz / K - k * nz / K);
  auto blocks_of = [&](int32_t p) {
    int64_t w = 0;
    for (int k = 0; k < K; ++k) w += tiles_of((k + 1) * nz / K - k * nz / K, ny, nx, T, p);
    return w;
  };
  return plan_tile_rows(block_slots(T), T, 4, static_cast<int32_t>(std::max<int64_t>(zmax, 4)),
                        blocks_of);
}

ccl_status launch_wave3d_tb(int32_t dtype, int32_t T, double r2, int32_t tile_planes,
                            const WaveChunkPlan *plans, int32_t nplans, hipStream_t stream) {
  if (T < 2 || T > CCL_MAX_DEPTH)
    return fail(CCL_E_INVALID, "temporally blocked 3D stencil needs T in 2..%d", CCL_MAX_DEPTH);
  const int NV = dtype_group(dtype);
  const int esize = dtype_bytes(dtype);
  if (esize == 0) return fail(CCL_E_INVALID, "unknown dtype %d", dtype);
  const uintptr_t amask = static_cast<uintptr_t>(NV * esize - 1);
  if (nplans < 1) return CCL_OK;
  const Box &D = plans[0].domain;
  for (int k = 0; k < nplans; ++k)
    for (int d = 0; d < 3; ++d)
      if (plans[k].domain.lo[d] != D.lo[d] || plans[k].domain.hi[d] != D.hi[d])
        return fail(CCL_E_INVALID, "chunks of one launch must share the domain");
  for (int d = 0; d < 3; ++d)
    if (!fits_i32(D.lo[d] - 64) || !fits_i32(D.hi[d] + 64))
      return fail(CCL_E_RANGE, "3D indices must fit in int32");
  for (int first = 0; first < nplans; first += kMaxChunksPerLaunch) {
    const int n = std::min(kMaxChunksPerLaunch, nplans - first);
    W3TArgs a;
    memset(&a, 0, sizeof(a));
    a.nchunks = n;
    a.r2f = static_cast<float>(r2);
    a.r2d = r2;
    a.gz0 = static_cast<int32_t>(D.lo[0]);
    a.gz1 = static_cast<int32_t>(D.hi[0]);
    a.gy0 = static_cast<int32_t>(D.lo[1]);
    a.gy1 = static_cast<int32_t>(D.hi[1]);
    a.gx0 = static_cast<int32_t>(D.lo[2]);
    a.gx1 = static_cast<int32_t>(D.hi[2]);
    if (tile_planes > 0) {
      a.tile_planes = tile_planes;
    } else {
      int64_t zmax = 0;
      for (int k = 0; k < n; ++k)
        zmax = std::max<int64_t>(zmax, plans[first + k].chunk.hi[0] - plans[first + k].chunk.lo[0]);
      auto blocks_of = [&](int32_t p) {
        int64_t w = 0;
        for (int k = 0; k < n; ++k) {
          const Box &cb = plans[first + k].chunk;
          w += tiles_of(cb.hi[0] - cb.lo[0], cb.hi[1] - cb.lo[1], cb.hi[2] - cb.lo[2], T, p, NV);
        }
        return w;
      };
      a.tile_planes = plan_tile_rows(block_slots(T, dtype), T, 4,
                                     static_cast<int32_t>(std::max<int64_t>(zmax, 4)), blocks_of);
    }
    int64_t tiles = 0;
    for (int k = 0; k < n; ++k) {
      const WaveChunkPlan &P = plans[first + k];
      W3TChunk &C = a.ch[k];
      C.in_prev = P.in_prev.base;
      C.in_cur = P.in_cur.base;
      C.out_prev = P.out_prev.base;
      C.out_cur = P.out_cur.base;
      const WaveField *fs[4] = {&P.in_prev, &P.in_cur, &P.out_prev, &P.out_cur};
      Field3 *gs[4] = {&C.ip, &C.ic, &C.op, &C.oc};
      // strip 0's patches start A columns left of the chunk, aligned down
      // to a multiple of NV relative to the u^n buffer so that every
      // thread's group of NV columns is one aligned vector access
      const int64_t A = tb_overlap(T, NV);
      const int64_t mis = (((P.chunk.lo[2] - A - P.in_cur.off[2]) % NV) + NV) % NV;
      const int64_t xs0 = P.chunk.lo[2] - A - mis;
      if (!fits_i32(xs0)) return fail(CCL_E_RANGE, "3D indices must fit in int32");
      C.xs0 = static_cast<int32_t>(xs0);
      for (int b = 0; b < 4; ++b) {
        ccl_status st = field3_of(*fs[b], gs[b]);
        if (st != CCL_OK) return st;
        if ((((xs0 - fs[b]->off[2]) % NV) + NV) % NV != 0 || fs[b]->pitch[0] % NV != 0 ||
            fs[b]->pitch[1] % NV != 0 || (reinterpret_cast<uintptr_t>(fs[b]->base) & amask) != 0)
          return fail(CCL_E_INVALID,
                      "chunk %d: 3D buffers must be %d-byte aligned with strides a multiple of "
                      "%d and the same region column offset modulo %d",
                      first + k, NV * esize, NV, NV);
      }
      box6(P.load_prev, C.lp);
      box6(P.load_cur, C.lc);
      C.cz0 = static_cast<int32_t>(P.chunk.lo[0]);
      C.cz1 = static_cast<int32_t>(P.chunk.hi[0]);
      C.cy0 = static_cast<int32_t>(P.chunk.lo[1]);
      C.cy1 = static_cast<int32_t>(P.chunk.hi[1]);
      C.cx0 = static_cast<int32_t>(P.chunk.lo[2]);
      C.cx1 = static_cast<int32_t>(P.chunk.hi[2]);
      const int64_t nz = P.chunk.hi[0] - P.chunk.lo[0];
      const int64_t ny = P.chunk.hi[1] - P.chunk.lo[1];
      const int64_t nx = P.chunk.hi[2] - (xs0 + A);  // output columns from strip 0's first
      C.nstrips = static_cast<int32_t>((nx + tb_out_cols(T, NV) - 1) / tb_out_cols(T, NV));
      C.nrowblk = static_cast<int32_t>((ny + tb_out_rows(T) - 1) / tb_out_rows(T));
      C.tile_begin = static_cast<int32_t>(tiles);
      tiles += tiles_of(nz, ny, nx, T, a.tile_planes, NV);
      if (tiles > INT32_MAX / 2) return fail(CCL_E_RANGE, "too many tiles");
    }
    a.total_tiles = static_cast<int32_t>(tiles);
    if (tiles == 0) continue;
    ccl_status st = launch_k(kernel_for(dtype, T), a, static_cast<int>(tiles), stream);
    if (st != CCL_OK) return st;
  }
  return CCL_OK;
}

}  // namespace ccl
