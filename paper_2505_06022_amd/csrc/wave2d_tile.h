// Device code of one 2D wave tile, shared by the chunked launch (wave2d.hip)
// and the batched persistent launch (batch.hip).
//
// Work unit: one wave (64 lanes) owns a tile = a strip of 64*NV columns (NV
// consecutive elements per lane: four floats, two doubles or four 16-bit
// values, one vector load each; see prec.h) and a segment of output rows.
// The wave streams down the rows: at iteration i it loads row i of u^n and
// row i-1 of u^{n-1}, then computes level 2 at row i-1, level 3 at row i-2,
// ..., level T+1 at row i-T, keeping the last three rows of every level in
// registers (rotating slots, so no row is moved between iterations).  North/south neighbours come from that register ring; west/east
// neighbours from the adjacent lane through DPP wave shifts (no LDS, no
// barriers).  A level-(k+1) value is only valid where its whole dependency
// cone was loaded, so strips overlap by NV*ceil(T/NV) columns on each side and
// segments re-read T rows above and below; outputs are written only for the
// valid interior.  Every cell value is produced by the same expression in
// the arithmetic type, so results are bitwise independent of tiling and
// chunking (and of T, where storage and arithmetic types agree).
//
// In place (T == 1 only): u^{n+1} overwrites u^{n-1}; each lane then reads
// u^{n-1} only at the cells it writes.  Otherwise u^{n+T-1} and u^{n+T} go to
// a second buffer pair, because neighbouring tiles still read the halo cells
// of the inputs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "prec.h"

namespace ccl {
namespace w2 {

// Rows loaded ahead of use, and rows per unrolled loop body.  The body is
// a whole number of turns of both the three-row ring and the prefetch
// slots, so its copy uu finds every level's newest row in ring slot uu % 3
// and its prefetched rows in slot uu % kPrefetch, and nothing is moved
// between iterations.  The out-of-place update holds its stores until the
// next body (see tile()), so within a body only loads are outstanding and
// each use waits for its own row's loads alone; the wait for everything
// outstanding comes once per body, at its head.  For float32 a 12-row body
// makes that wait 4x rarer than a 3-row one (measured on the 8192 x 8192
// share with 32-row tiles: 28.6 ms per 1000 steps at T = 8 against 30.5,
// 32.0 against 34.6 at T = 7, 37.0 against 39.6 at T = 6), at 12 held rows
// per level pair (210 VGPRs at T = 8, two waves per SIMD).  The float64 and
// 16-bit types keep 3-row bodies (PR::kBody; 12 rows made them slower), as
// does the in-place T = 1 update, which stores as it goes.
#ifndef CCL_W2_PREFETCH
#define CCL_W2_PREFETCH 3
#endif
constexpr int kPrefetch = CCL_W2_PREFETCH;
template <class PR>
__host__ __device__ constexpr int unroll_of(bool in_place) {
  return in_place ? 3 : PR::kBody;
}


// Overlap columns per side and output columns per strip for depth T, with
// NV columns per lane.
__host__ __device__ constexpr int overlap(int T, int NV = 4) { return NV * ((T + NV - 1) / NV); }
__host__ __device__ constexpr int strip_width(int T, int NV = 4) {
  return 64 * NV - 2 * overlap(T, NV);
}

struct Chunk {
  const void *in_prev;
  const void *in_cur;
  void *out_prev;
  void *out_cur;
  int32_t ip_y0, ip_x0, ip_pitch;
  int32_t ic_y0, ic_x0, ic_pitch;
  int32_t op_y0, op_x0, op_pitch;
  int32_t oc_y0, oc_x0, oc_pitch;
  int32_t lp_y0, lp_y1, lp_x0, lp_x1;  // loadable box of in_prev (region ∩ domain)
  int32_t lc_y0, lc_y1, lc_x0, lc_x1;  // loadable box of in_cur
  int32_t cy0, cy1, cx0, cx1;          // chunk (output) box
  int32_t xs0;                         // first column of strip 0
  int32_t nstrips;
  int32_t tile_begin;
  int32_t push_begin, push_end;        // this chunk's entries of the launch's pushes
};

// A halo push: rows of this launch's output that another chunk's next
// launch reads from its own buffers.  The launch stores them there too, so
// no separate exchange is needed before the next block of steps.  Rows
// [cr0, cr1) of u^{n+T} go to `cur`, rows [pr0, pr1) of u^{n+T-1} to `prev`
// (the other chunk's output buffers of this launch, which nothing reads
// during it); the columns are the source chunk's, which for a split along
// rows are the whole domain width.
struct Push {
  void *cur;
  void *prev;
  int32_t cur_y0, cur_x0, cur_pitch;
  int32_t prev_y0, prev_x0, prev_pitch;
  int32_t cr0, cr1, pr0, pr1;
};

// The pushes of one chunk, passed to the tile by value (kept in scalar
// registers): a chunk of a split along rows has at most two neighbours.
constexpr int kMaxPush = 2;
struct PushSet {
  int32_t n;
  Push p[kMaxPush];
};

struct Domain {
  int32_t gy0, gy1, gx0, gx1;  // zero outside
};

__device__ __forceinline__ float fma_(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return fma(a, b, c); }

// One cell: s = (N + S) + (W + E); lap = s - 4C; u+ = fma(r2, lap, 2C - P).
// 4C and 2C are exact in binary floating point, so s - 4C and 2C - P are
// each the exact value rounded once, which is what the fma forms below
// compute: the result is bitwise the same as the separate multiply and
// subtract, with two fewer instructions.
template <class F>
__device__ __forceinline__ F cell(F n, F s, F w, F e, F c, F p, F r2) {
  const F sum = (n + s) + (w + e);
  const F lap = fma_(F(-4), c, sum);
  return fma_(r2, lap, fma_(F(2), c, -p));
}

// One lane group's update; west / east neighbours of the group's outer
// columns come from the adjacent lanes.
template <class PR>
__device__ __forceinline__ Vec<typename PR::F, PR::NV> step_group(
    const Vec<typename PR::F, PR::NV> &n, const Vec<typename PR::F, PR::NV> &c,
    const Vec<typename PR::F, PR::NV> &s, const Vec<typename PR::F, PR::NV> &p,
    typename PR::F r2) {
  constexpr int NV = PR::NV;
  using F = typename PR::F;
  const F left = dpp_move<0x138>(c.v[NV - 1]);   // wave_shr:1
  const F right = dpp_move<0x130>(c.v[0]);       // wave_shl:1
  Vec<F, NV> o;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const F w = i == 0 ? left : c.v[i > 0 ? i - 1 : 0];
    const F e = i == NV - 1 ? right : c.v[i < NV - 1 ? i + 1 : 0];
    o.v[i] = cell(n.v[i], s.v[i], w, e, c.v[i], p.v[i], r2);
  }
  return o;
}

template <class F, int NV>
__device__ __forceinline__ Vec<F, NV> zero_vec() {
  Vec<F, NV> z;
#pragma unroll
  for (int i = 0; i < NV; ++i) z.v[i] = F(0);
  return z;
}

// Which of the lane's NV columns [xl, xl+NV) lie in [x0, x1).  Columns are
// grouped in aligned NV-tuples relative to the buffer, and a buffer's pitch
// is a multiple of NV that covers its extent, so a group that meets
// [x0, x1) is always inside the allocated row.
struct Cols {
  bool any;
  bool m[4];
};

template <int NV = 4>
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

typedef float f4v __attribute__((ext_vector_type(4)));

// The first and the last aligned group of NV columns (aligned relative to
// the buffer's first column bx0) that meet [x0, x1), a non-empty range of
// the buffer's columns; such groups lie inside the allocated row.
template <int NV = 4>
__device__ __forceinline__ int clamp_group(int xl, int x0, int x1, int bx0) {
  const int g0 = x0 - ((x0 - bx0) & (NV - 1));
  const int g1 = (x1 - 1) - ((x1 - 1 - bx0) & (NV - 1));
  return min(max(xl, g0), g1);
}

// Loads a group unconditionally: the caller passes a row and a group that
// the buffer holds (clamped into the loadable box), so the load needs no
// branch and stays in flight until its value is used; cells outside the box
// are zeroed later by mask_group, where the value is consumed.  STREAM
// marks data read once: u^{n-1} in the in-place T = 1 update, where a
// nontemporal load keeps it from displacing the u^n rows that neighbouring
// tiles re-read from cache (15% faster than a cached load).  For T > 1 the
// u^{n-1} rows in the overlap of vertically adjacent segments are read
// twice too, and a cached load is 1-2% faster at T = 7, 8.
template <class PR, bool STREAM>
__device__ __forceinline__ typename PR::Raw load_group(const void *base, int32_t by0, int32_t bx0,
                                                       int32_t pitch, int row, int xg) {
  using Raw = typename PR::Raw;
  const Raw *p = reinterpret_cast<const Raw *>(static_cast<const typename PR::E *>(base) +
                                               static_cast<int64_t>(row - by0) * pitch +
                                               (xg - bx0));
  return STREAM ? __builtin_nontemporal_load(p) : *p;
}

// Loads a group as 32-bit words at the device-coherent level (relaxed
// agent-scope atomic loads, which do not hit the vector L1): used to read
// back what this lane has just stored.
template <class PR>
__device__ __forceinline__ typename PR::Raw load_group_coherent(const void *base, int32_t by0,
                                                                int32_t bx0, int32_t pitch,
                                                                int row, int xg) {
  using Raw = typename PR::Raw;
  constexpr int kWords = sizeof(Raw) / 4;
  static_assert(sizeof(Raw) % 4 == 0, "groups are whole 32-bit words");
  const uint32_t *p = reinterpret_cast<const uint32_t *>(
      static_cast<const typename PR::E *>(base) + static_cast<int64_t>(row - by0) * pitch +
      (xg - bx0));
  uint32_t w[kWords];
#pragma unroll
  for (int i = 0; i < kWords; ++i)
    w[i] = __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  Raw r;
  __builtin_memcpy(&r, w, sizeof(Raw));
  return r;
}

// Widens a loaded group, zero outside the loadable box: the row
// (wave-uniform) and the lane's columns.
template <class PR>
__device__ __forceinline__ Vec<typename PR::F, PR::NV> mask_group(const typename PR::Raw &r,
                                                                  bool row_ok, const Cols &c) {
  Vec<typename PR::F, PR::NV> v;
#pragma unroll
  for (int i = 0; i < PR::NV; ++i)
    v.v[i] = (row_ok && c.m[i]) ? PR::widen(r[i]) : typename PR::F(0);
  return v;
}

// Stores the lane's group of `row` where the output mask allows, narrowed
// to the storage type (nontemporal: nothing in this launch reads it back).
// Partial groups occur only at a chunk's left or right edge; their other
// columns are halo cells of this chunk's own buffer that no wave writes
// during the launch, so they are read and written back unchanged (one
// vector store).
template <class PR>
__device__ __forceinline__ void store_group(void *base, int32_t by0, int32_t bx0, int32_t pitch,
                                            int row, int xl, const Cols &c,
                                            const Vec<typename PR::F, PR::NV> &v) {
  using Raw = typename PR::Raw;
  if (!c.any) return;
  Raw *p = reinterpret_cast<Raw *>(static_cast<typename PR::E *>(base) +
                                   static_cast<int64_t>(row - by0) * pitch + (xl - bx0));
  Raw w;
#pragma unroll
  for (int i = 0; i < PR::NV; ++i) w[i] = PR::narrow(v.v[i]);
  if (!all_of<PR::NV>(c)) {
    const Raw o = *p;
#pragma unroll
    for (int i = 0; i < PR::NV; ++i) w[i] = c.m[i] ? w[i] : o[i];
  }
  __builtin_nontemporal_store(w, p);
}

template <class F, int NV>
__device__ __forceinline__ Vec<F, NV> force_zero(Vec<F, NV> v, bool row_in, const Cols &d) {
#pragma unroll
  for (int i = 0; i < NV; ++i) v.v[i] = (row_in && d.m[i]) ? v.v[i] : F(0);
  return v;
}

// Advances one tile (segment `seg`, strip `strip` of chunk C) by T steps.
// Strips are 64*NV columns wide and overlap their neighbours by A columns on
// each side (A >= T, a multiple of NV); each writes SW = 64*NV - 2A columns.
// The descriptors are copied into registers once: read through a reference
// inside the loop, they would be reloaded after every store (the compiler
// cannot rule out that a store aliases them).
template <class PR, int T, bool IN_PLACE, int U = unroll_of<PR>(IN_PLACE)>
__device__ __forceinline__ void tile(const Chunk &Cref, const Domain &Dref, typename PR::F r2,
                                     int tile_rows, int seg, int strip, int lane, int A,
                                     const PushSet &PSref = PushSet{0, {}}) {
  constexpr int kUnroll = U;
  static_assert(U % kPrefetch == 0 && U % 3 == 0, "whole turns of the ring and the prefetch");
  constexpr int NV = PR::NV;
  using F = typename PR::F;
  using V = Vec<F, NV>;
  using Raw = typename PR::Raw;
  const Chunk C = Cref;
  const Domain D = Dref;
  const int SW = 64 * NV - 2 * A;
  const int y0 = C.cy0 + seg * tile_rows;
  const int y1 = min(C.cy1, y0 + tile_rows);
  const int xs = C.xs0 + strip * SW;
  const int xl = xs + NV * lane;
  const int vx0 = max(C.cx0, xs + A);
  const int vx1 = min(C.cx1, xs + A + SW);

  const Cols dom = cols_of<NV>(xl, D.gx0, D.gx1);
  const Cols out = cols_of<NV>(xl, vx0, vx1);
  const Cols lc = cols_of<NV>(xl, C.lc_x0, C.lc_x1);
  // In place, u^{n-1} is read only where this lane writes.
  const int lpy0 = IN_PLACE ? max(C.lp_y0, y0) : C.lp_y0;
  const int lpy1 = IN_PLACE ? min(C.lp_y1, y1) : C.lp_y1;
  const Cols lp = cols_of<NV>(xl, IN_PLACE ? max(C.lp_x0, vx0) : C.lp_x0,
                              IN_PLACE ? min(C.lp_x1, vx1) : C.lp_x1);

  // a strip whose columns all lie in the domain needs no column mask
  const bool interior_cols = xs >= D.gx0 && xs + 64 * NV <= D.gx1;

  // halo pushes that meet this tile's output rows (only tiles at the edges
  // of a chunk have any; wave-uniform); made after the streaming loop
  const PushSet PS = PSref;
  bool has_push = false;
#pragma unroll
  for (int p = 0; p < kMaxPush; ++p) {
    const Push &P = PS.p[p];
    has_push = has_push ||
               (p < PS.n && ((P.cr0 < y1 && P.cr1 > y0) || (P.pr0 < y1 && P.pr1 > y0)));
  }

  // ring[k][s]: the last three rows of level k in rotating slots; at the
  // unrolled copy uu the newest row goes to slot uu%3, the middle one is in
  // (uu+2)%3 and the oldest in (uu+1)%3
  V ring[T][3];
#pragma unroll
  for (int k = 0; k < T; ++k) ring[k][0] = ring[k][1] = ring[k][2] = zero_vec<F, NV>();

  const int first = y0 - T;
  const int nrows = (y1 - y0) + 2 * T;
  // loads go to rows and groups clamped into the loadable box (never empty:
  // it holds the chunk's rows and columns), masks apply on use
  const int xgc = clamp_group<NV>(xl, C.lc_x0, C.lc_x1, C.ic_x0);
  const int xgp = clamp_group<NV>(xl, IN_PLACE ? max(C.lp_x0, vx0) : C.lp_x0,
                                  IN_PLACE ? min(C.lp_x1, vx1) : C.lp_x1, C.ip_x0);
  auto row_c = [&](int r) { return min(max(r, C.lc_y0), C.lc_y1 - 1); };
  auto row_p = [&](int r) { return min(max(r, lpy0), lpy1 - 1); };
  Raw q1[kPrefetch], q0[kPrefetch];
#pragma unroll
  for (int u = 0; u < kPrefetch; ++u) {
    q1[u] = load_group<PR, false>(C.in_cur, C.ic_y0, C.ic_x0, C.ic_pitch,
                                  row_c(first + u), xgc);
    q0[u] = load_group<PR, IN_PLACE>(C.in_prev, C.ip_y0, C.ip_x0, C.ip_pitch,
                                     row_p(first + u - 1), xgp);
  }

  // Stores are issued one loop iteration late.  One counter tracks both
  // loads and stores on this target, and stores and loads may complete out
  // of order, so the compiler's wait for a load at the loop head also waits
  // for every store issued before it; a store issued at the top of the
  // previous iteration has had a whole iteration of arithmetic to complete
  // (measured: +7-8% at T = 8 on an 8192 x 8192 share).  Issuing the next
  // iteration's loads at its top as well was slower than this alone.  The
  // in-place T = 1 update keeps its stores in place.
  constexpr bool DEFER = !IN_PLACE;
  // level-T rows of the previous iteration (u^{n+T}, u^{n+T-1}) and whether
  // each lies in the tile's output rows (wave-uniform)
  V d1[kUnroll], d0[kUnroll];
  bool dok[kUnroll];
#pragma unroll
  for (int uu = 0; uu < kUnroll; ++uu) dok[uu] = false;
  int jlast = 0;

  // kUnroll rows per loop iteration (a multiple of the ring length): the
  // compiler waits for all outstanding memory operations once per
  // iteration, at the loop head, so a longer body exposes that latency
  // less often.
  //
  // Warm-up: level k at streamed row m (row first + m - k) feeds a stored
  // output only if m >= 2k (level k is needed on rows [first + k, ...): the
  // outputs' dependency cone narrows by one row per level), so the bodies
  // at the start of the stream (the first, and those after it that lie
  // wholly within the first 2T rows) are separate copies in which level k
  // is computed only at rows m >= 2k, a compile-time condition, and the
  // levels above a skipped one are skipped too.  Everything a computed
  // level reads was computed (rows m-2..m of level k-1, and m-2 >= 2(k-1)),
  // so the stored values are unchanged; the skipped work is T(T+1) of the
  // tile's T * nrows level-rows, or nearly (at T = 8 with 12-row bodies,
  // 66 of the 72 rows the warm-up wastes: one copy of the body covers rows
  // 0..11).
  constexpr int kWarmBodies = 2 * T > kUnroll ? 1 + (2 * T - kUnroll) / kUnroll : 1;
  // JB: the compile-time first row of a warm-up body, -1 in the steady loop
  auto body = [&](auto jb_tag, int jb) {
    constexpr int JB = decltype(jb_tag)::value;
    if constexpr (DEFER && JB != 0) {
#pragma unroll
      for (int uu = 0; uu < kUnroll; ++uu) {
        if (dok[uu]) {
          const int r = first + jb - kUnroll + uu - T;
          store_group<PR>(C.out_cur, C.oc_y0, C.oc_x0, C.oc_pitch, r, xl, out, d1[uu]);
          store_group<PR>(C.out_prev, C.op_y0, C.op_x0, C.op_pitch, r, xl, out, d0[uu]);
        }
      }
    }
#pragma unroll
    for (int uu = 0; uu < kUnroll; ++uu) {
      const int u = uu % kPrefetch;  // prefetch slot
      const int NEW = uu % 3, MID = (uu + 2) % 3, OLD = (uu + 1) % 3;
      const int i = first + jb + uu;  // row of level 0 arriving now
      ring[0][NEW] = mask_group<PR>(q1[u], i >= C.lc_y0 && i < C.lc_y1, lc);
      V pv = mask_group<PR>(q0[u], i - 1 >= lpy0 && i - 1 < lpy1, lp);
      q1[u] = load_group<PR, false>(C.in_cur, C.ic_y0, C.ic_x0, C.ic_pitch,
                                    row_c(i + kPrefetch), xgc);
      q0[u] = load_group<PR, IN_PLACE>(C.in_prev, C.ip_y0, C.ip_x0, C.ip_pitch,
                                       row_p(i + kPrefetch - 1), xgp);
#pragma unroll
      for (int k = 1; k <= T; ++k) {
        if (JB >= 0 && JB + uu < 2 * k) break;  // not needed yet (compile-time)
        const int r = i - k;  // row of level k computed now
        V nv = step_group<PR>(ring[k - 1][OLD], ring[k - 1][MID], ring[k - 1][NEW], pv, r2);
        const bool row_in = r >= D.gy0 && r < D.gy1;  // wave-uniform
        if (!(row_in && interior_cols)) nv = force_zero(nv, row_in, dom);
        if (k < T) {
          pv = ring[k - 1][OLD];
          ring[k < T ? k : 0][NEW] = nv;
        } else if constexpr (DEFER) {
          dok[uu] = r >= y0 && r < y1;
          d1[uu] = nv;
          d0[uu] = ring[T - 1][MID];
        } else if (r >= y0 && r < y1) {
          store_group<PR>(C.out_cur, C.oc_y0, C.oc_x0, C.oc_pitch, r, xl, out, nv);
          if (!IN_PLACE)
            store_group<PR>(C.out_prev, C.op_y0, C.op_x0, C.op_pitch, r, xl, out,
                            ring[T - 1][MID]);
        }
      }
    }
  };
  auto warm_up = [&](auto self, auto jb_tag) {
    constexpr int JB = decltype(jb_tag)::value;
    if (JB == 0 || JB < nrows) {  // the first body always runs (nrows > 0)
      body(jb_tag, JB);
      jlast = JB;
    }
    if constexpr (JB / kUnroll + 1 < kWarmBodies)
      self(self, std::integral_constant<int, JB + kUnroll>());
  };
  warm_up(warm_up, std::integral_constant<int, 0>());
  for (int jb = kWarmBodies * kUnroll; jb < nrows; jb += kUnroll) {
    body(std::integral_constant<int, -1>(), jb);
    jlast = jb;
  }
  if constexpr (DEFER) {
#pragma unroll
    for (int uu = 0; uu < kUnroll; ++uu) {
      if (dok[uu]) {
        const int r = first + jlast + uu - T;
        store_group<PR>(C.out_cur, C.oc_y0, C.oc_x0, C.oc_pitch, r, xl, out, d1[uu]);
        store_group<PR>(C.out_prev, C.op_y0, C.op_x0, C.op_pitch, r, xl, out, d0[uu]);
      }
    }
  }
  if (has_push) {
    // the pushed rows are this lane's own groups of its output buffers, just
    // stored: read them back and store them into the other chunks' buffers
    // (at most 2T rows per field, in the tiles at the edges of a chunk
    // only).  A lane reads only what it stored itself, so it is enough to
    // wait until its stores have completed and to read at the device-coherent
    // level (an agent-scope fence would also write back the whole L2 of the
    // XCD: measured 8% slower launches)
    __builtin_amdgcn_s_waitcnt(0);
    // all of a push's rows (at most T) are read first and then stored, so
    // the reads overlap
    auto copy_rows = [&](const void *src, int32_t sy0, int32_t sx0, int32_t spitch, void *dst,
                         int32_t dy0, int32_t dx0, int32_t dpitch, int r0, int r1) {
      Raw buf[T];
#pragma unroll
      for (int j = 0; j < T; ++j)
        if (r0 + j < r1) buf[j] = load_group_coherent<PR>(src, sy0, sx0, spitch, r0 + j, xl);
#pragma unroll
      for (int j = 0; j < T; ++j)
        if (r0 + j < r1)
          store_group<PR>(dst, dy0, dx0, dpitch, r0 + j, xl, out, mask_group<PR>(buf[j], true, out));
    };
    if (out.any) {
#pragma unroll
      for (int p = 0; p < kMaxPush; ++p) {
        const Push &P = PS.p[p];
        if (p >= PS.n) continue;
        // a push covers at most T rows of the chunk, and a tile's share of
        // them is one contiguous range
        const int c0 = max(y0, P.cr0), c1 = min(y1, P.cr1);
        if (c0 < c1)
          copy_rows(C.out_cur, C.oc_y0, C.oc_x0, C.oc_pitch, P.cur, P.cur_y0, P.cur_x0,
                    P.cur_pitch, c0, min(c1, c0 + T));
        const int p0 = max(y0, P.pr0), p1 = min(y1, P.pr1);
        if (!IN_PLACE && p0 < p1)
          copy_rows(C.out_prev, C.op_y0, C.op_x0, C.op_pitch, P.prev, P.prev_y0, P.prev_x0,
                    P.prev_pitch, p0, min(p1, p0 + T));
      }
    }
  }
}

// Maps a block index so that consecutive logical blocks land on the same
// XCD (blocks are dispatched to the 8 XCDs round-robin); neighbouring tiles
// then share an L2 for the rows and columns they both read.
__device__ __forceinline__ int xcd_block(int bid, int nblocks) {
  const int q = nblocks >> 3, r = nblocks & 7;
  const int xcd = bid & 7, idx = bid >> 3;
  return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + idx;
}

}  // namespace w2
}  // namespace ccl
