// Many independent 2D grids stepped by one persistent launch, captured in a
// HIP graph (or, with CCL_BATCH_PER_GRID, by each grid's own ccl_wave_step
// sequence captured in the same way).
//
// Every grid is cut into the same 2D tiles as the chunked launch (a strip of
// 256 columns by a segment of rows, processed by one wave with the code in
// wave2d_tile.h) and advanced in blocks of T steps, double-buffered: block b
// reads buffer pair b%2 and writes the other.  A tile's block b may start
// once the 3x3 tiles around it (itself included) have finished block b-1:
// that covers both the halo it reads (T <= segment rows, A <= strip width)
// and the cells of pair (b+1)%2 it overwrites, which those tiles read during
// block b-1.  Each tile keeps a progress counter (blocks done), released
// after its stores; waiters acquire it before reading.
//
// Work order: a single queue holds all (block, grid, tile) items sorted by
// block, then depth class, then grid, then tile.  (A queue ordered grid by
// grid, so that the resident waves would pipeline one grid's blocks while
// its buffers stay cache-resident, was measured 20x slower: the blocks of
// one grid depend on each other, so at any time only about one block of
// one grid can run and the other waves hold queue items they must wait on.)  (Stepping small groups of grids whose
// buffers fit in the 256 MB Infinity Cache block by block was measured 5x
// slower: a block of two grids is too little work to hide the hand-off
// between consecutive blocks.)  Waves pop items with an atomic counter.  An
// item of block b depends only on items of the same grid at block b-1, all
// of which sit earlier in the queue and were popped by waves that are
// running, so every wait ends without any assumption about how many waves
// are resident.  A wait also ends after a time limit (an error flag is
// raised and all waves drain the queue without computing), so the launch
// always completes.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "ccl_internal.h"
#include "wave2d_tile.h"

namespace ccl {
namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kThreads = 64 * kWavesPerBlock;


struct GridDev {
  float *buf[4];
  int32_t ny, nx, pitch;
  int32_t T, last_T, A;
  int32_t tile_rows, nstrips, nsegs, nblocks;
  int32_t counter_base;
  float r2;
};

// The queue is a list of segments, one per (block, depth class): the tiles
// of the class's grids that have that block, grids [g0, gend) of the sorted
// list (each class is sorted by block count, descending, so the grids still
// active at a block are a prefix of the class).
struct BatchTables {
  const GridDev *grids;          // by depth class, then nblocks descending
  const int32_t *prefix_tiles;   // [ngrids + 1] tiles before each grid
  const int32_t *seg_start;      // [nseg + 1] queue index of each segment's first item
  const int32_t *seg_block;      // [nseg] the segment's block
  const int32_t *seg_g0;         // [nseg] its first grid
  const int32_t *seg_gend;       // [nseg] one past its last grid
  int32_t *counters;             // per tile: blocks completed
  int32_t *ctl;                  // [0] queue head, [1] error flag
  const int64_t *wait_ticks;     // wall-clock ticks a wait may last
  int32_t total;
  int32_t nseg;
  int32_t ncounters;
};

__global__ __launch_bounds__(256) void batch_reset_kernel(int32_t *counters, int32_t n,
                                                          int32_t *ctl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) counters[i] = 0;
  if (i < 2) ctl[i] = 0;
}

__device__ __forceinline__ int upper_index(const int32_t *a, int lo, int n, int32_t v) {
  // largest i in [lo, n) with a[i] <= v (a ascending, a[lo] <= v)
  int hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a[mid] <= v)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Counter and flag reads while waiting are relaxed device-scope loads
// (they read the coherent value without cache maintenance); the single
// acquire fence after the last wait makes the neighbours' data visible.  An
// acquire load per poll would invalidate the XCD's L2 on every iteration
// of every waiting wave, evicting the rows the other waves stream.
__device__ __forceinline__ int32_t load_relaxed(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits until counters[idx] >= want.  Returns false if the batch's error
// flag is (or gets) raised, or the wait limit passes (then raises it).
__device__ bool wait_for(const BatchTables &t, int idx, int32_t want, uint64_t t0,
                         int64_t limit) {
  while (load_relaxed(&t.counters[idx]) < want) {
    if (load_relaxed(&t.ctl[1]) != 0) return false;
    if (static_cast<int64_t>(wall_clock64() - t0) > limit) {
      __hip_atomic_store(&t.ctl[1], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return true;
}

// Runs tile<tb> for the block's depth tb (<= TMAX, the largest depth of any
// grid in the batch, which bounds the registers the kernel needs).
template <int TMAX, int T = 1>
__device__ __forceinline__ void dispatch_depth(int tb, const w2::Chunk &C, const w2::Domain &D,
                                               float r2, int tile_rows, int seg, int strip,
                                               int lane, int A) {
  if (tb == T || T == TMAX) {
    // 3 rows per loop body: the kernel holds the code of every depth up to
    // TMAX, and 12-row bodies would take it to one wave per SIMD
    w2::tile<P32, T, false, 3>(C, D, r2, tile_rows, seg, strip, lane, A);
  } else if constexpr (T < TMAX) {
    dispatch_depth<TMAX, T + 1>(tb, C, D, r2, tile_rows, seg, strip, lane, A);
  }
}

template <int TMAX>
__global__ __launch_bounds__(kThreads) void batch_kernel(const BatchTables t) {
  const int lane = threadIdx.x & 63;
  const int64_t limit = *t.wait_ticks;
  for (;;) {
    int32_t q = 0;
    if (lane == 0) q = __hip_atomic_fetch_add(&t.ctl[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    q = __builtin_amdgcn_readfirstlane(q);
    if (q >= t.total) break;
    const int sg = upper_index(t.seg_start, 0, t.nseg, q);
    const int b = t.seg_block[sg];
    const int g0 = t.seg_g0[sg];
    const int32_t local = q - t.seg_start[sg] + t.prefix_tiles[g0];
    const int g = upper_index(t.prefix_tiles, g0, t.seg_gend[sg], local);
    const GridDev G = t.grids[g];
    const int tl = local - t.prefix_tiles[g];
    const int seg = tl / G.nstrips;
    const int strip = tl - seg * G.nstrips;

    bool ok = load_relaxed(&t.ctl[1]) == 0;
    if (ok && b > 0) {
      const uint64_t t0 = wall_clock64();
      for (int ds = -1; ds <= 1 && ok; ++ds) {
        const int s2 = seg + ds;
        if (s2 < 0 || s2 >= G.nsegs) continue;
        for (int dx = -1; dx <= 1 && ok; ++dx) {
          const int x2 = strip + dx;
          if (x2 < 0 || x2 >= G.nstrips) continue;
          ok = wait_for(t, G.counter_base + s2 * G.nstrips + x2, b, t0, limit);
        }
      }
    }
    if (!ok) continue;  // error raised: drain the queue without computing
    // the neighbours' block b-1 (written on any XCD) is visible from here
    if (b > 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");

    const int set = b & 1;
    w2::Chunk C;
    C.in_prev = G.buf[2 * set];
    C.in_cur = G.buf[2 * set + 1];
    C.out_prev = G.buf[2 * (1 - set)];
    C.out_cur = G.buf[2 * (1 - set) + 1];
    C.ip_y0 = C.ic_y0 = C.op_y0 = C.oc_y0 = 0;
    C.ip_x0 = C.ic_x0 = C.op_x0 = C.oc_x0 = 0;
    C.ip_pitch = C.ic_pitch = C.op_pitch = C.oc_pitch = G.pitch;
    C.lp_y0 = C.lc_y0 = C.cy0 = 0;
    C.lp_y1 = C.lc_y1 = C.cy1 = G.ny;
    C.lp_x0 = C.lc_x0 = C.cx0 = 0;
    C.lp_x1 = C.lc_x1 = C.cx1 = G.nx;
    C.xs0 = -G.A;
    C.nstrips = G.nstrips;
    C.tile_begin = 0;
    C.push_begin = C.push_end = 0;  // the batch's tiles share no buffers
    const w2::Domain D{0, G.ny, 0, G.nx};
    const int tb = (b == G.nblocks - 1) ? G.last_T : G.T;
    dispatch_depth<TMAX>(tb, C, D, G.r2, G.tile_rows, seg, strip, lane, G.A);
    // publish: one release fence (every lane's stores complete and written
    // back device-wide), then the counter moves to b+1
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane == 0)
      __hip_atomic_store(&t.counters[G.counter_base + tl], b + 1, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <int TMAX>
const void *batch_kernel_ptr() {
  return reinterpret_cast<const void *>(&batch_kernel<TMAX>);
}

}  // namespace

struct BatchImpl {
  int32_t ngrids = 0;
  int32_t tmax = 1;
  int32_t flags = 0;
  std::vector<ccl_batch_grid> grids;  // caller order
  std::vector<int32_t> nblocks;       // caller order
  void *dev = nullptr;                // one allocation for all tables
  BatchTables tables{};
  int blocks = 0;                     // persistent grid size
  int counter_blocks = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t *wait_ticks_dev = nullptr;
  std::vector<int32_t> final_prev, final_cur;  // CCL_BATCH_PER_GRID: buffer roles at the end
};

// CCL_BATCH_PER_GRID: every grid stepped by its own ccl_wave_step call (one
// chunk, its own T and tile rows), one grid after another, so that each
// grid's buffers stay cache-resident across its T-blocks.
static ccl_status enqueue_per_grid(BatchImpl *B, hipStream_t s) {
  for (int g = 0; g < B->ngrids; ++g) {
    const ccl_batch_grid &G = B->grids[g];
    if (G.steps == 0) continue;
    ccl_chunk ch;
    memset(&ch, 0, sizeof(ch));
    ch.dims = 2;
    ch.range[0] = ch.global_range[0] = G.ny;
    ch.range[1] = ch.global_range[1] = G.nx;
    ccl_chunk_buffer b[4];
    for (int k = 0; k < 4; ++k) {
      memset(&b[k], 0, sizeof(b[k]));
      b[k].base = G.buf[k];
      b[k].region.dims = 2;
      b[k].region.range[0] = G.ny;
      b[k].region.range[1] = G.nx;
      b[k].pitch[0] = G.pitch;
      b[k].pitch[1] = 1;
    }
    ccl_wave_params p;
    memset(&p, 0, sizeof(p));
    p.dims = 2;
    p.r2 = G.r2;
    p.temporal_depth = G.temporal_depth;
    p.tile_rows = G.tile_rows;
    ccl_status st = ccl_wave_step(&p, 1, &ch, &b[0], &b[1], &b[2], &b[3], G.steps, s);
    if (st != CCL_OK) return st;
  }
  return CCL_OK;
}

// The counter reset and the persistent kernel over tables `t`.
static ccl_status launch_persistent(const BatchTables &t, int tmax, int blocks,
                                    int counter_blocks, hipStream_t s) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3(counter_blocks), dim3(256), 0, s, t.counters,
                     t.ncounters, t.ctl);
  ccl_status st = hip_check(hipGetLastError(), "batch_reset_kernel launch");
  if (st != CCL_OK) return st;
  TimedLaunch tl(CCL_KERNEL_STENCIL, s);
  switch (tmax) {
    case 1: hipLaunchKernelGGL(batch_kernel<1>, dim3(blocks), dim3(kThreads), 0, s, t); break;
    case 2: hipLaunchKernelGGL(batch_kernel<2>, dim3(blocks), dim3(kThreads), 0, s, t); break;
    case 4: hipLaunchKernelGGL(batch_kernel<4>, dim3(blocks), dim3(kThreads), 0, s, t); break;
    default: hipLaunchKernelGGL(batch_kernel<8>, dim3(blocks), dim3(kThreads), 0, s, t); break;
  }
  return hip_check(hipGetLastError(), "batch_kernel launch");
}

static ccl_status enqueue_batch(BatchImpl *B, hipStream_t s) {
  if (B->flags & CCL_BATCH_PER_GRID) return enqueue_per_grid(B, s);
  return launch_persistent(B->tables, B->tmax, B->blocks, B->counter_blocks, s);
}

static void release(BatchImpl *B) {
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
  if (B->dev) (void)hipFree(B->dev);
  delete B;
}

}  // namespace ccl

using namespace ccl;

struct ccl_batch {
  BatchImpl *impl;
};

namespace ccl {

// Checks the grids and fills their device descriptors (tile rows still 0
// where automatic); tmax is rounded up to a depth the kernel is built for.
static ccl_status validate_grids(int32_t ngrids, const ccl_batch_grid *grids,
                                 std::vector<GridDev> *gd_out, std::vector<int32_t> *nblk_out,
                                 int *tmax_out) {
  if (ngrids > 0 && !grids) return fail(CCL_E_INVALID, "NULL argument");
  if (ngrids < 1) return fail(CCL_E_INVALID, "ngrids=%d < 1", ngrids);
  std::vector<GridDev> &gd = *gd_out;
  std::vector<int32_t> &nblk = *nblk_out;
  gd.assign(ngrids, GridDev{});
  nblk.assign(ngrids, 0);
  int tmax = 1;
  for (int g = 0; g < ngrids; ++g) {
    const ccl_batch_grid &G = grids[g];
    if (G.ny < 1 || G.nx < 1 || G.ny > (1 << 30) || G.nx > (1 << 30))
      return fail(CCL_E_INVALID, "grid %d: extents out of range", g);
    if (G.pitch < G.nx || (G.pitch % 4) != 0 || G.pitch > (int64_t(1) << 31) / 2)
      return fail(CCL_E_INVALID, "grid %d: pitch must be >= nx and a multiple of 4", g);
    if (G.steps < 0) return fail(CCL_E_INVALID, "grid %d: steps < 0", g);
    if (G.temporal_depth < 1 || G.temporal_depth > CCL_MAX_DEPTH)
      return fail(CCL_E_INVALID, "grid %d: temporal depth %d not in 1..8", g, G.temporal_depth);
    if (!std::isfinite(G.r2) || G.r2 < 0.0f) return fail(CCL_E_INVALID, "grid %d: bad r2", g);
    if (G.tile_rows != 0 && G.tile_rows < G.temporal_depth)
      return fail(CCL_E_INVALID, "grid %d: tile_rows must be >= T", g);
    for (int k = 0; k < 4; ++k)
      if (!G.buf[k] || (reinterpret_cast<uintptr_t>(G.buf[k]) & 15u) != 0)
        return fail(CCL_E_INVALID, "grid %d: buf[%d] NULL or not 16-byte aligned", g, k);
    GridDev &D = gd[g];
    for (int k = 0; k < 4; ++k) D.buf[k] = G.buf[k];
    D.ny = static_cast<int32_t>(G.ny);
    D.nx = static_cast<int32_t>(G.nx);
    D.pitch = static_cast<int32_t>(G.pitch);
    D.T = G.temporal_depth;
    D.A = w2::overlap(D.T);
    D.tile_rows = G.tile_rows;  // 0: planned later
    D.nstrips = static_cast<int32_t>((G.nx + w2::strip_width(D.T) - 1) / w2::strip_width(D.T));
    D.nblocks = (G.steps + D.T - 1) / D.T;
    D.last_T = G.steps - D.T * (D.nblocks > 0 ? D.nblocks - 1 : 0);
    D.r2 = G.r2;
    nblk[g] = D.nblocks;
    tmax = std::max(tmax, D.T);
  }
  *tmax_out = tmax <= 1 ? 1 : tmax <= 2 ? 2 : tmax <= 4 ? 4 : 8;
  return CCL_OK;
}

// Host-side plan of one persistent launch: the queue order, tile counters
// and the grid size.
struct PersistentPlan {
  int32_t tmax = 1;
  int blocks = 1;
  std::vector<GridDev> sorted;  // by depth class, then block count
  std::vector<int32_t> prefix, seg_start, seg_block, seg_g0, seg_gend;
  int64_t counters = 0, total = 0;
  int32_t nseg = 0;
};

static ccl_status plan_persistent(std::vector<GridDev> gd, int tmax, PersistentPlan *P) {
  const int ngrids = static_cast<int>(gd.size());
  // persistent grid: as many blocks as fit on the device at once
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  e = e ? e : hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const void *kfn = tmax == 1   ? batch_kernel_ptr<1>()
                    : tmax == 2 ? batch_kernel_ptr<2>()
                    : tmax == 4 ? batch_kernel_ptr<4>()
                                : batch_kernel_ptr<8>();
  e = e ? e : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, kThreads, 0);
  if (e != hipSuccess) return hip_check(e, "occupancy query");
  const int blocks = std::max(1, cus * std::max(1, per_cu));
  const int64_t slots = static_cast<int64_t>(blocks) * kWavesPerBlock;

  // order: by depth class (T descending), then block count, descending
  // (stable).  Within a block the queue then holds one depth class after
  // another, so the waves running at any moment execute the same tile code
  // (mixing depths cost ~15%: each depth is its own unrolled loop)
  std::vector<int> order(ngrids);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return gd[a].T != gd[b].T ? gd[a].T > gd[b].T : gd[a].nblocks > gd[b].nblocks;
  });
  // automatic tile rows: the largest candidate that still gives every
  // resident wave a tile of the first block; at least max(8, T)
  {
    // (each item costs a dependency wait and a cache write-back, so fewer,
    // taller tiles win while every wave still has one: 64 grids measured
    // 57.5 ms at 512 rows, 60.4 at 256, 70.3 at 1024 with too few items)
    static const int32_t kRowsCand[] = {512, 256, 128, 64, 32, 16, 8};
    int32_t chosen = 0;
    for (int32_t r : kRowsCand) {
      int64_t items = 0;
      for (const GridDev &D : gd) {
        const int32_t rr = D.tile_rows > 0 ? D.tile_rows : std::max(r, std::max(8, D.T));
        items += static_cast<int64_t>((D.ny + rr - 1) / rr) * D.nstrips;
      }
      chosen = r;
      if (items >= slots) break;
    }
    for (GridDev &D : gd)
      if (D.tile_rows == 0) D.tile_rows = std::max(chosen, std::max(8, D.T));
  }
  int64_t counters = 0;
  for (int g = 0; g < ngrids; ++g) {
    GridDev &D = gd[g];
    D.nsegs = static_cast<int32_t>((D.ny + D.tile_rows - 1) / D.tile_rows);
    D.counter_base = static_cast<int32_t>(counters);
    counters += static_cast<int64_t>(D.nstrips) * D.nsegs;
    if (counters > INT32_MAX / 4) return fail(CCL_E_RANGE, "too many tiles");
  }
  P->sorted.assign(ngrids, GridDev{});
  P->prefix.assign(ngrids + 1, 0);
  for (int i = 0; i < ngrids; ++i) {
    P->sorted[i] = gd[order[i]];
    P->prefix[i + 1] = P->prefix[i] + P->sorted[i].nstrips * P->sorted[i].nsegs;
  }
  // queue segments: (block, depth class) -> the class's grids still active
  // (a prefix of the class, which is sorted by block count)
  std::vector<int32_t> cls;  // first grid of each depth class, then ngrids
  for (int i = 0; i < ngrids; ++i)
    if (i == 0 || P->sorted[i].T != P->sorted[i - 1].T) cls.push_back(i);
  cls.push_back(ngrids);
  int32_t max_blocks = 0;
  for (const GridDev &D : P->sorted) max_blocks = std::max(max_blocks, D.nblocks);
  P->seg_start.clear();
  P->seg_block.clear();
  P->seg_g0.clear();
  P->seg_gend.clear();
  int64_t total = 0;
  for (int b = 0; b < max_blocks; ++b) {
    for (size_t c = 0; c + 1 < cls.size(); ++c) {
      int a = cls[c];
      while (a < cls[c + 1] && P->sorted[a].nblocks > b) ++a;
      if (a == cls[c]) continue;
      P->seg_start.push_back(static_cast<int32_t>(total));
      P->seg_block.push_back(b);
      P->seg_g0.push_back(cls[c]);
      P->seg_gend.push_back(a);
      total += P->prefix[a] - P->prefix[cls[c]];
      if (total > INT32_MAX / 2) return fail(CCL_E_RANGE, "batch queue too long");
    }
  }
  P->nseg = static_cast<int32_t>(P->seg_block.size());
  P->seg_start.push_back(static_cast<int32_t>(total));
  P->counters = counters;
  P->total = total;
  P->tmax = tmax;
  P->blocks = total == 0 ? 1 : blocks;
  return CCL_OK;
}

// Byte offsets of the tables in one contiguous device range:
// grids | prefix | segment tables | counters | ctl | wait ticks.
struct TableLayout {
  size_t grids, prefix, sstart, sblock, sg0, sgend, count, ctl, wait, bytes;
};

static TableLayout layout_of(const PersistentPlan &P) {
  auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
  const size_t ng = P.sorted.size();
  const size_t nsg = static_cast<size_t>(std::max(P.nseg, 1));
  TableLayout L;
  L.grids = 0;
  L.prefix = al(L.grids + sizeof(GridDev) * ng);
  L.sstart = al(L.prefix + sizeof(int32_t) * (ng + 1));
  L.sblock = al(L.sstart + sizeof(int32_t) * (nsg + 1));
  L.sg0 = al(L.sblock + sizeof(int32_t) * nsg);
  L.sgend = al(L.sg0 + sizeof(int32_t) * nsg);
  L.count = al(L.sgend + sizeof(int32_t) * nsg);
  L.ctl = al(L.count + sizeof(int32_t) * static_cast<size_t>(std::max<int64_t>(P.counters, 1)));
  L.wait = al(L.ctl + sizeof(int32_t) * 2);
  L.bytes = al(L.wait + sizeof(int64_t));
  return L;
}

constexpr int64_t kDefaultWaitTicks = int64_t(100000000) * 10;  // 10 s of the 100 MHz clock

// The tables' bytes as they must appear in device memory (counters and
// control words zero; the reset kernel clears them again before each run).
static void write_tables(const PersistentPlan &P, const TableLayout &L, char *h) {
  memset(h, 0, L.bytes);
  auto put = [&](size_t off, const void *src, size_t n) {
    if (n > 0) memcpy(h + off, src, n);
  };
  put(L.grids, P.sorted.data(), sizeof(GridDev) * P.sorted.size());
  put(L.prefix, P.prefix.data(), sizeof(int32_t) * P.prefix.size());
  put(L.sstart, P.seg_start.data(), sizeof(int32_t) * P.seg_start.size());
  put(L.sblock, P.seg_block.data(), sizeof(int32_t) * P.seg_block.size());
  put(L.sg0, P.seg_g0.data(), sizeof(int32_t) * P.seg_g0.size());
  put(L.sgend, P.seg_gend.data(), sizeof(int32_t) * P.seg_gend.size());
  put(L.wait, &kDefaultWaitTicks, sizeof(int64_t));
}

// The kernel's view of tables laid out by `L` at device address `d`.
static BatchTables tables_at(const PersistentPlan &P, const TableLayout &L, char *d) {
  BatchTables t;
  t.grids = reinterpret_cast<const GridDev *>(d + L.grids);
  t.prefix_tiles = reinterpret_cast<const int32_t *>(d + L.prefix);
  t.seg_start = reinterpret_cast<const int32_t *>(d + L.sstart);
  t.seg_block = reinterpret_cast<const int32_t *>(d + L.sblock);
  t.seg_g0 = reinterpret_cast<const int32_t *>(d + L.sg0);
  t.seg_gend = reinterpret_cast<const int32_t *>(d + L.sgend);
  t.counters = reinterpret_cast<int32_t *>(d + L.count);
  t.ctl = reinterpret_cast<int32_t *>(d + L.ctl);
  t.wait_ticks = reinterpret_cast<const int64_t *>(d + L.wait);
  t.total = static_cast<int32_t>(P.total);
  t.nseg = P.nseg;
  t.ncounters = static_cast<int32_t>(P.counters);
  return t;
}

static int counter_blocks_of(const PersistentPlan &P) {
  return static_cast<int>((std::max<int64_t>(P.counters, 2) + 255) / 256);
}

}  // namespace ccl

extern "C" ccl_status ccl_batch_create(int32_t ngrids, const ccl_batch_grid *grids,
                                       int32_t flags, ccl_batch **out) {
  clear_error();
  if (!out || (ngrids > 0 && !grids)) return fail(CCL_E_INVALID, "NULL argument");
  if ((flags & ~(CCL_BATCH_NO_GRAPH | CCL_BATCH_PER_GRID)) != 0)
    return fail(CCL_E_INVALID, "unknown flags");
  std::vector<GridDev> gd;
  std::vector<int32_t> nblk;
  int tmax = 1;
  ccl_status st = validate_grids(ngrids, grids, &gd, &nblk, &tmax);
  if (st != CCL_OK) return st;

  BatchImpl *B = nullptr;
  if (flags & CCL_BATCH_PER_GRID) {
    B = new BatchImpl();
    B->ngrids = ngrids;
    B->flags = flags;
    B->grids.assign(grids, grids + ngrids);
    B->nblocks = nblk;
    // the roles ccl_wave_step's rotation leaves: T = 1 blocks swap u_prev
    // and u_cur, T > 1 blocks swap each with its second buffer
    for (int g = 0; g < ngrids; ++g) {
      int up = 0, uc = 1, wp = 2, wc = 3;
      for (int done = 0; done < grids[g].steps;) {
        const int tb = std::min(grids[g].temporal_depth, grids[g].steps - done);
        if (tb == 1) {
          std::swap(up, uc);
        } else {
          std::swap(up, wp);
          std::swap(uc, wc);
        }
        done += tb;
      }
      B->final_prev.push_back(up);
      B->final_cur.push_back(uc);
    }
  } else {
    PersistentPlan P;
    st = plan_persistent(gd, tmax, &P);
    if (st != CCL_OK) return st;
    B = new BatchImpl();
    B->ngrids = ngrids;
    B->tmax = tmax;
    B->flags = flags;
    B->grids.assign(grids, grids + ngrids);
    B->nblocks = nblk;
    const TableLayout L = layout_of(P);
    st = hip_check(hipMalloc(&B->dev, L.bytes), "hipMalloc(batch tables)");
    if (st != CCL_OK) {
      delete B;
      return fail(CCL_E_NOMEM, "batch tables: %s", ccl_last_error());
    }
    std::vector<char> host(L.bytes);
    write_tables(P, L, host.data());
    hipError_t e = hipMemcpy(B->dev, host.data(), L.bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      release(B);
      return hip_check(e, "hipMemcpy(batch tables)");
    }
    char *d = static_cast<char *>(B->dev);
    B->tables = tables_at(P, L, d);
    B->wait_ticks_dev = reinterpret_cast<int64_t *>(d + L.wait);
    B->counter_blocks = counter_blocks_of(P);
    B->blocks = P.blocks;
  }

  hipError_t e = hipSuccess;
  if (!(flags & CCL_BATCH_NO_GRAPH)) {
    e = hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking);
    e = e ? e : hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      release(B);
      return hip_check(e, "graph capture start");
    }
    st = enqueue_batch(B, B->cap_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(B->cap_stream, &graph);
    B->graph = graph;
    if (st != CCL_OK || e != hipSuccess) {
      release(B);
      return st != CCL_OK ? st : hip_check(e, "graph capture end");
    }
    e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      release(B);
      return hip_check(e, "hipGraphInstantiate");
    }
  }
  ccl_batch *h = new ccl_batch{B};
  *out = h;
  return CCL_OK;
}

extern "C" ccl_status ccl_batch_run(ccl_batch *b, void *hip_stream) {
  clear_error();
  if (!b || !b->impl) return fail(CCL_E_INVALID, "NULL batch");
  BatchImpl *B = b->impl;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (B->exec) {
    TimedLaunch tl(CCL_KERNEL_BATCH, s);
    return hip_check(hipGraphLaunch(B->exec, s), "hipGraphLaunch");
  }
  return enqueue_batch(B, s);
}

extern "C" ccl_status ccl_batch_check(ccl_batch *b, void *hip_stream) {
  clear_error();
  if (!b || !b->impl) return fail(CCL_E_INVALID, "NULL batch");
  BatchImpl *B = b->impl;
  ccl_status st = hip_check(hipStreamSynchronize(static_cast<hipStream_t>(hip_stream)),
                            "hipStreamSynchronize");
  if (st != CCL_OK) return st;
  if (B->flags & CCL_BATCH_PER_GRID) return CCL_OK;  // no waits to time out
  int32_t ctl[2] = {0, 0};
  st = hip_check(hipMemcpy(ctl, B->tables.ctl, sizeof(ctl), hipMemcpyDeviceToHost),
                 "hipMemcpy(batch status)");
  if (st != CCL_OK) return st;
  if (ctl[1] != 0) return fail(CCL_E_TIMEOUT, "a tile's dependency wait passed its limit");
  return CCL_OK;
}

extern "C" ccl_status ccl_batch_set_wait_limit(ccl_batch *b, int64_t microseconds) {
  clear_error();
  if (!b || !b->impl) return fail(CCL_E_INVALID, "NULL batch");
  if (microseconds < 0) return fail(CCL_E_INVALID, "negative wait limit");
  if (b->impl->flags & CCL_BATCH_PER_GRID) return CCL_OK;  // nothing waits
  const int64_t ticks = microseconds * 100;  // 100 MHz wall clock
  return hip_check(hipMemcpy(b->impl->wait_ticks_dev, &ticks, sizeof(ticks),
                             hipMemcpyHostToDevice),
                   "hipMemcpy(wait limit)");
}

extern "C" ccl_status ccl_batch_result(const ccl_batch *b, int32_t grid, int32_t *prev_buf,
                                       int32_t *cur_buf) {
  clear_error();
  if (!b || !b->impl || !prev_buf || !cur_buf) return fail(CCL_E_INVALID, "NULL argument");
  if (grid < 0 || grid >= b->impl->ngrids) return fail(CCL_E_INVALID, "grid %d out of range", grid);
  if (b->impl->flags & CCL_BATCH_PER_GRID) {
    *prev_buf = b->impl->final_prev[grid];
    *cur_buf = b->impl->final_cur[grid];
    return CCL_OK;
  }
  const int set = b->impl->nblocks[grid] & 1;
  *prev_buf = 2 * set;
  *cur_buf = 2 * set + 1;
  return CCL_OK;
}

extern "C" ccl_status ccl_batch_destroy(ccl_batch *b) {
  clear_error();
  if (!b) return CCL_OK;
  if (b->impl) release(b->impl);
  delete b;
  return CCL_OK;
}

// ---- the persistent run without device allocation --------------------------
//
// The tables, tile counters and control words of one persistent run live in
// `scratch`, a fixed file-scope device array: every GPU the library runs on
// holds its own copy until the process ends.  In host code the array's name
// stands for no device address, so host code uses only the address
// hipGetSymbolAddress returns for the current device, taken once per device.

static __device__ __align__(256) unsigned char scratch[CCL_BATCH_STATIC_BYTES];

namespace ccl {
namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_dev[kMaxScratchDevices] = {};

// The current device's copy of `scratch` (its address is looked up on the
// first call made with that device current).
ccl_status scratch_of_current_device(char **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_check(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxScratchDevices)
    return fail(CCL_E_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxScratchDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_check(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(CCL_E_HIP, "hipGetSymbolAddress(scratch) gave NULL");
    g_scratch_dev[dev] = static_cast<char *>(ptr);
  }
  *out = g_scratch_dev[dev];
  return CCL_OK;
}

}  // namespace
}  // namespace ccl

extern "C" ccl_status ccl_batch_run_static(int32_t ngrids, const ccl_batch_grid *grids,
                                           int32_t *prev_buf, int32_t *cur_buf,
                                           int32_t *wait_failed, void *hip_stream) {
  clear_error();
  std::vector<GridDev> gd;
  std::vector<int32_t> nblk;
  int tmax = 1;
  ccl_status st = validate_grids(ngrids, grids, &gd, &nblk, &tmax);
  if (st != CCL_OK) return st;
  PersistentPlan P;
  st = plan_persistent(gd, tmax, &P);
  if (st != CCL_OK) return st;
  const TableLayout L = layout_of(P);
  if (L.bytes > sizeof(scratch))
    return fail(CCL_E_RANGE,
                "the batch needs %zu bytes of tables and counters, more than the %zu of the "
                "static array (fewer grids or taller tiles fit)",
                L.bytes, sizeof(scratch));
  char *d = nullptr;
  st = scratch_of_current_device(&d);
  if (st != CCL_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // tables from host memory (the copy is ordered on `s`; the host copy may
  // go once the call returns), then the counters and control words cleared
  // by the reset kernel inside launch_persistent
  std::vector<char> host(L.bytes);
  write_tables(P, L, host.data());
  st = hip_check(hipMemcpyAsync(d, host.data(), L.bytes, hipMemcpyHostToDevice, s),
                 "hipMemcpyAsync(batch tables)");
  if (st != CCL_OK) return st;
  const BatchTables t = tables_at(P, L, d);
  st = launch_persistent(t, P.tmax, P.blocks, counter_blocks_of(P), s);
  if (st != CCL_OK) return st;
  for (int g = 0; g < ngrids; ++g) {
    const int set = nblk[g] & 1;
    if (prev_buf) prev_buf[g] = 2 * set;
    if (cur_buf) cur_buf[g] = 2 * set + 1;
  }
  if (wait_failed) {
    st = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (st != CCL_OK) return st;
    int32_t ctl[2] = {0, 0};
    st = hip_check(hipMemcpy(ctl, t.ctl, sizeof(ctl), hipMemcpyDeviceToHost),
                   "hipMemcpy(batch status)");
    if (st != CCL_OK) return st;
    *wait_failed = ctl[1] != 0 ? 1 : 0;
    if (ctl[1] != 0) return fail(CCL_E_TIMEOUT, "a tile's dependency wait passed its limit");
  }
  return CCL_OK;
}
