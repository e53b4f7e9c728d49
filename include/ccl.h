/*
 * ccl.h -- C ABI of libccl: chunked range-mapper stencils on MI355X (gfx950).
 *
 * The execution model is the one the paper describes for Celerity (section
 * 3, second listing and the paragraph after it): a data-parallel kernel runs
 * over an N-D index range; the range is split into chunks, one per device;
 * each accessor carries a range mapper that ties a chunk of the kernel's
 * range to the region of a buffer the chunk reads or writes; the regions a
 * chunk needs but does not own are inferred from the mappers and copied in
 * before the chunk runs.  Here every chunk is device-local (its own buffer
 * in the one GPU's memory), so the inferred transfers are device-to-device
 * copies.  The chunk kernel is a 2D five-point / 3D seven-point leapfrog
 * wave-equation stencil; SAXPY (the paper's first listing, section 2) is
 * exported for bandwidth calibration, and device energy is read the way the
 * paper's SYnergy queue exposes it (section 4, third listing).
 *
 * Conventions for every entry point
 *   - Return value: CCL_OK (0) or a negative ccl_status; out-parameters are
 *     written only on success.  ccl_last_error() returns a thread-local
 *     message describing the most recent failure on the calling thread.
 *   - No exception ever crosses this ABI.
 *   - Memory: the caller owns all field memory (device pointers obtained
 *     from hipMalloc or a framework allocator) and all streams.  The library
 *     allocates only the opaque objects returned by *_create functions,
 *     released by the matching *_destroy.
 *   - Streams: `hip_stream` is a hipStream_t passed as void* (NULL = the
 *     default stream).  Device work is enqueued asynchronously and the call
 *     returns; launch errors are reported synchronously as CCL_E_HIP, faults
 *     during execution surface at the caller's next synchronisation.
 *   - Index spaces are global: chunk offsets, buffer regions and boxes are
 *     given in the coordinates of the buffer (Celerity's virtual buffer),
 *     dimension 0 slowest.  All integer extents are int64.
 *   - Layout of a chunk buffer: element (i_0, ..., i_{D-1}) of the global
 *     index space lives at base + sum_d (i_d - region.offset[d]) * pitch[d]
 *     elements, with pitch[D-1] == 1 (row-major, innermost contiguous).
 */
#ifndef CCL_H
#define CCL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ccl_status;

enum {
  CCL_OK = 0,
  CCL_E_INVALID = -1,     /* bad argument: NULL, dims, counts, alignment   */
  CCL_E_RANGE = -2,       /* an index box falls outside what is allowed    */
  CCL_E_HIP = -3,         /* a HIP runtime call failed                     */
  CCL_E_UNSUPPORTED = -4, /* feature not available (e.g. energy counter)   */
  CCL_E_NOMEM = -5,       /* host or device allocation failed              */
  CCL_E_STATE = -6,       /* object used in the wrong state                */
  CCL_E_TIMEOUT = -7      /* a bounded device-side wait gave up            */
};

#define CCL_MAX_DIMS 3
#define CCL_MAX_CHUNKS 64      /* chunks per ccl_wave_step / exchange call  */
#define CCL_MAX_DEPTH 8        /* largest temporal depth T                  */

/* An N-D box of indices: [offset[d], offset[d] + range[d]) for d < dims.
 * Entries at d >= dims are ignored. */
typedef struct {
  int32_t dims;
  int64_t offset[CCL_MAX_DIMS];
  int64_t range[CCL_MAX_DIMS];
} ccl_subrange;

/* One chunk of a kernel's execution range.  `offset/range` is the chunk,
 * `global_offset/global_range` the whole range it was split from (the
 * parallel_for range).  For the wave stencil the global range is also the
 * problem domain: cells outside it hold zero (homogeneous Dirichlet). */
typedef struct {
  int32_t dims;
  int64_t offset[CCL_MAX_DIMS];
  int64_t range[CCL_MAX_DIMS];
  int64_t global_offset[CCL_MAX_DIMS];
  int64_t global_range[CCL_MAX_DIMS];
} ccl_chunk;

/* Range mappers (section 3: the accessor's range mapper ties a chunk of the
 * kernel's range to the data it touches).  ONE_TO_ONE: the chunk touches
 * exactly its own indices (the mapper of the paper's second listing).
 * NEIGHBORHOOD: the chunk grown by extent[d] on both sides of every
 * dimension (a stencil's read set).  ALL: the whole buffer.  FIXED: the box
 * [offset, offset + extent), whatever the chunk (data every chunk reads,
 * such as a coefficient table).  SLICE: the chunk, taken whole along
 * dimension `dim` (a row or column reduction's read set).  Every region is
 * clipped to the buffer's index range. */
typedef enum {
  CCL_MAP_ONE_TO_ONE = 0,
  CCL_MAP_NEIGHBORHOOD = 1,
  CCL_MAP_ALL = 2,
  CCL_MAP_FIXED = 3,
  CCL_MAP_SLICE = 4
} ccl_mapper_kind;

typedef struct {
  int32_t kind;                   /* a ccl_mapper_kind                      */
  int64_t extent[CCL_MAX_DIMS];   /* NEIGHBORHOOD: growth per side, >= 0;
                                     FIXED: extent of the box, >= 0         */
  int64_t offset[CCL_MAX_DIMS];   /* FIXED: first index of the box          */
  int32_t dim;                    /* SLICE: the dimension taken whole       */
} ccl_range_mapper;

/* A chunk's slice of one buffer in device memory (caller-owned). */
typedef struct {
  void *base;                     /* device address of region.offset   */
  ccl_subrange region;            /* global indices held               */
  int64_t pitch[CCL_MAX_DIMS];    /* element strides; pitch[dims-1]==1 */
} ccl_chunk_buffer;

/* One inferred transfer: box (global indices) owned by chunk `owner` and
 * needed by chunk `reader`. */
typedef struct {
  int32_t owner;
  int32_t reader;
  ccl_subrange box;
} ccl_transfer;

/* Element types of the wave fields.  F32 and F64 compute in their own
 * precision.  BF16 (bfloat16) and F16 (IEEE binary16) store the fields in
 * 16 bits and compute in float32: a launch widens what it loads, applies its
 * T steps in float32 and rounds the two levels it stores to nearest, ties
 * to even, so their results depend on T (not on chunking or tiling). */
enum {
  CCL_DTYPE_F32 = 0,
  CCL_DTYPE_F64 = 1,
  CCL_DTYPE_BF16 = 2,
  CCL_DTYPE_F16 = 3
};

/* Wave-stencil parameters. */
typedef struct {
  int32_t dims;              /* 2 or 3                                       */
  double r2;                 /* (c dt / dx)^2; stable for r2 <= 1/dims; used
                                as given for F64, rounded once to float32
                                for the other element types                  */
  int32_t temporal_depth;    /* T in 1..CCL_MAX_DEPTH steps per HBM pass     */
  int32_t tile_rows;         /* rows (2D) / planes (3D) per wave tile, 0=auto*/
  int32_t flags;             /* reserved, must be 0                          */
  int32_t dtype;             /* CCL_DTYPE_*: element type of every buffer    */
} ccl_wave_params;

/* ----------------------------------------------------------------------- */

/* Library version string (static storage). */
const char *ccl_version(void);

/* Message for the most recent failure on this thread ("" if none). */
const char *ccl_last_error(void);

/* Split a kernel range into chunks (section 3: a kernel is split across all
 * available devices).  Along `split_dim`, chunk k of `nchunks` covers
 * [o + floor(k n / K), o + floor((k+1) n / K)) where o, n are the range's
 * offset and extent there; other dimensions are whole.  Chunks are disjoint,
 * cover the range, and differ in size by at most one.
 *   range        : the kernel range (dims in 1..3, range[d] >= 1)
 *   chunks_out   : caller array of `nchunks` entries
 * Errors: INVALID (NULL, dims, nchunks < 1, split_dim), RANGE (nchunks larger
 * than the extent along split_dim). */
ccl_status ccl_split_range(const ccl_subrange *range, int32_t nchunks,
                           int32_t split_dim, ccl_chunk *chunks_out);

/* Split a kernel range into a grid of chunks: counts[d] pieces along every
 * dimension d (section 3: the kernel is split across the available devices;
 * a block split keeps each chunk's halo short in every dimension).  Chunk
 * (k_0, ..., k_{D-1}) covers, along each d, [o + floor(k_d n / K_d),
 * o + floor((k_d + 1) n / K_d)) with o, n the range's offset and extent and
 * K_d = counts[d]; chunks are numbered row-major over the grid (the last
 * dimension fastest).  With one count above 1 this is ccl_split_range along
 * that dimension.
 *   counts     : range->dims entries, each >= 1
 *   chunks_out : caller array of counts[0] * ... * counts[D-1] entries
 * Errors: INVALID (NULL, dims, a count < 1), RANGE (a count larger than the
 * extent along its dimension). */
ccl_status ccl_split_grid(const ccl_subrange *range, const int32_t *counts,
                          ccl_chunk *chunks_out);

/* Region of a buffer that a chunk accesses through a range mapper (section
 * 3: the range mapper ties a chunk of the execution range to its data
 * requirements).  Every region is clipped to [0, buffer_range).
 *   buffer_range : extent of the (virtual) buffer, dims entries
 * Errors: INVALID (NULL, dims mismatch, unknown kind, negative extent, SLICE
 * dim outside [0, dims)). */
ccl_status ccl_region_of(const ccl_chunk *chunk, const ccl_range_mapper *mapper,
                         const int64_t *buffer_range, ccl_subrange *region_out);

/* Transfers a set of chunks needs before its kernel can run (section 3: the
 * range mappers are used to infer the data transfers): for every ordered
 * pair (owner k, reader j != k), region_of(chunk j, mapper) intersected with
 * chunk k, when non-empty.  Writes at most `capacity` entries and the total
 * count to *count (call with capacity 0 to size the array).
 * Errors: INVALID, RANGE (count exceeds capacity: *count still written). */
ccl_status ccl_transfers(int32_t nchunks, const ccl_chunk *chunks,
                         const ccl_range_mapper *mapper,
                         const int64_t *buffer_range, ccl_transfer *out,
                         int32_t capacity, int32_t *count);

/* Perform the inferred transfers between device-local chunk buffers: every
 * box that ccl_transfers derives for `mapper` is copied from bufs[owner] to
 * bufs[reader], all boxes in one kernel launch on `hip_stream`.
 *   bufs       : one buffer per chunk; bufs[k].region must contain chunk k
 *                and every box chunk k reads
 *   elem_bytes : element size, a multiple of 2 (2 = bfloat16 / binary16,
 *                4 = float, 8 = double); bases aligned to 4 bytes (2 for
 *                2-byte elements)
 * Errors: INVALID, RANGE (a box outside a buffer's region), HIP. */
ccl_status ccl_halo_exchange(int32_t nchunks, const ccl_chunk *chunks,
                             const ccl_range_mapper *mapper,
                             const ccl_chunk_buffer *bufs, int32_t elem_bytes,
                             void *hip_stream);

/* Pack boxes of chunk buffers into one contiguous staging buffer, box after
 * box, each box row-major (what a sender hands to an interconnect), and the
 * inverse.  Box b is read from / written to srcs[b] / dsts[b]; `staging`
 * must hold sum of box sizes * elem_bytes bytes.  One launch each.
 * Errors: INVALID, RANGE (box outside the buffer's region), HIP. */
ccl_status ccl_halo_pack(int32_t nboxes, const ccl_subrange *boxes,
                         const ccl_chunk_buffer *srcs, int32_t elem_bytes,
                         void *staging, void *hip_stream);
ccl_status ccl_halo_unpack(int32_t nboxes, const ccl_subrange *boxes,
                           const ccl_chunk_buffer *dsts, int32_t elem_bytes,
                           const void *staging, void *hip_stream);

/* Advance the leapfrog wave equation by `nsteps` steps over all chunks.
 *
 * Per step, every cell of the domain (the chunks' global range) gets
 *   2D: s = (u[i-1][j] + u[i+1][j]) + (u[i][j-1] + u[i][j+1]); lap = s - 4u
 *   3D: s = ((u[z-1] + u[z+1]) + (u[y-1] + u[y+1])) + (u[x-1] + u[x+1]);
 *       lap = s - 6u
 *   u_next = fma(r2, lap, 2u - u_prev)    (round-to-nearest, in float64 for
 *                                          F64 and float32 otherwise)
 * with zero outside the domain; the buffers hold elements of p->dtype.  Work proceeds in blocks of T =
 * temporal_depth steps (the last block may be shorter): before each block
 * the halos are exchanged as ccl_halo_exchange does with NEIGHBORHOOD(T) for
 * u_cur and NEIGHBORHOOD(T-1) for u_prev, then one launch advances every
 * chunk T steps.
 *
 *   chunks          : nchunks chunks of one range (from ccl_split_range or
 *                     any disjoint cover), dims == p->dims
 *   u_prev, u_cur   : per chunk, the buffers holding u^{n-1} and u^n; their
 *                     regions must contain the chunk grown by T-1 and T
 *                     (clipped to the domain) respectively
 *   w_prev, w_cur   : per chunk, a second pair of buffers of the same
 *                     geometry, needed when T > 1 (may be NULL when T == 1,
 *                     where u^{n+1} overwrites u^{n-1} in place)
 *   On return the four descriptor arrays have been rotated so that u_cur
 *   describes u^{n+nsteps} and u_prev u^{n+nsteps-1}; buffer contents in the
 *   other pair are unspecified.  Results are bitwise independent of the
 *   chunking and tile_rows, and for F32 and F64 of T too (BF16 and F16
 *   round what each block stores, so their results depend on T).
 * Alignment: every base 16-byte aligned (8-byte for BF16 and F16), pitch[0]
 * (and pitch[1] in 3D) a multiple of 4 elements (2 for F64).
 * Errors: INVALID, RANGE, HIP. */
ccl_status ccl_wave_step(const ccl_wave_params *p, int32_t nchunks,
                         const ccl_chunk *chunks, ccl_chunk_buffer *u_prev,
                         ccl_chunk_buffer *u_cur, ccl_chunk_buffer *w_prev,
                         ccl_chunk_buffer *w_cur, int32_t nsteps,
                         void *hip_stream);

/* Cumulative energy drawn by GPU `device` (HIP ordinal), in joules, with
 * the semantics of the paper's device-level energy query (section 4, third
 * listing); a kernel's energy is the difference of two reads around it.
 * If hip_stream is not NULL it is synchronised first.  The timestamp is the
 * counter's own, in nanoseconds.  Backed by the amd-smi energy accumulator.
 * Errors: INVALID, UNSUPPORTED (no working energy counter), HIP. */
ccl_status ccl_energy_read(int32_t device, void *hip_stream, double *joules,
                           uint64_t *timestamp_ns);

/* Name of the energy backend in use for `device` after its first read:
 * "amdsmi-energy-counter", "amdsmi-power-integrated" (socket power sampled
 * every 5 ms and integrated, where the accumulator is not exposed), "fake"
 * (forced by CCL_ENERGY_BACKEND=fake, for host-only tests), "unsupported"
 * or "unprobed".  Static storage. */
const char *ccl_energy_backend(int32_t device);

/* ---- Generic chunked parallel_for ----------------------------------------
 * One data-parallel function over the chunks of a kernel range, with
 * accessors that carry a range mapper and an access mode: the paper's
 * second listing (section 3), where SAXPY's three accessors use the
 * one_to_one mapper, the kernel is split across the devices and the range
 * mappers tell the runtime which transfers must precede each chunk. */
enum {
  CCL_ACCESS_READ = 1,
  CCL_ACCESS_WRITE = 2,
  CCL_ACCESS_READ_WRITE = 3
};

typedef struct {
  ccl_range_mapper mapper;        /* chunk -> region of this buffer it touches */
  int32_t mode;                   /* CCL_ACCESS_*                              */
  int64_t buffer_range[CCL_MAX_DIMS]; /* the buffer's index range [0, range)   */
  const ccl_chunk_buffer *bufs;   /* one float32 buffer per chunk (caller-owned
                                     device memory); bufs[k].region holds chunk
                                     k and region_of(chunk k, mapper)          */
} ccl_accessor;

enum {
  CCL_FN_SAXPY = 0,      /* accessors x (read), y (read), z (write):
                            z[i] = fma(a, x[i], y[i])                        */
  CCL_FN_SUM_ALONG = 1   /* accessors x (read; its mapper's region spans the
                            range along `dim`, e.g. SLICE(dim) or ALL), out
                            (write): out[i] = x[i with i_dim = lo] + ... +
                            x[i with i_dim = hi - 1], summed in index order
                            from 0 in float32, lo/hi the range's bounds       */
};

typedef struct {
  int32_t fn;    /* CCL_FN_*                        */
  float a;       /* CCL_FN_SAXPY: the scalar        */
  int32_t dim;   /* CCL_FN_SUM_ALONG: the dimension */
} ccl_kernel_fn;

/* Runs `fn` at every index of every chunk.  Before the launch, for every
 * readable accessor whose mapper reaches beyond the chunk, the part of
 * region_of(chunk j, mapper) that chunk k owns (its chunk box) is copied
 * from bufs[k] to bufs[j], as ccl_halo_exchange does; each chunk's own cells
 * of a readable buffer must hold the data on entry.  Written accessors must
 * use ONE_TO_ONE (the functions write only at their own index).  All work
 * is enqueued on `hip_stream`: one copy launch, then one launch per 8
 * chunks.
 *   chunks    : nchunks chunks of one range (ccl_split_range, ccl_split_grid
 *               or any disjoint cover)
 *   acc       : naccessors accessors, in the order the function lists them
 * Errors: INVALID (NULL, unknown function, wrong accessor count or modes, a
 * written accessor with another mapper, bad buffers), RANGE (a buffer region
 * lacks its mapper's region, the range outside a buffer), HIP. */
ccl_status ccl_parallel_for(const ccl_kernel_fn *fn, int32_t nchunks, const ccl_chunk *chunks,
                            int32_t naccessors, const ccl_accessor *acc, void *hip_stream);

/* z[i] = fma(a, x[i], y[i]) for i < n, float32: the kernel of the paper's
 * first listing (section 2), used to measure achievable HBM bandwidth.
 * x, y, z: device arrays of n floats, 16-byte aligned.  Errors: INVALID, HIP. */
ccl_status ccl_saxpy(int64_t n, float a, const float *x, const float *y,
                     float *z, void *hip_stream);

/* Discrete energy of the leapfrog scheme, computed on the device:
 *   E^{n+1/2} = sum_i (a_i - b_i)^2 + r2 * sum_{edges (p,q)} (a_p - a_q)(b_p - b_q)
 * with a = u^{n+1}, b = u^n, over every edge of the dims-D grid, the edges
 * to the zero cells just outside the domain included.  In exact arithmetic
 * the update conserves it (take the update's inner product with
 * u^{n+1} - u^{n-1}; the discrete Laplacian is symmetric), and it is
 * positive under the step-size condition r2 < 1/dims, so it monitors a
 * run's stability and rounding drift.  The scheme is the chunk kernel that
 * stands in for the paper's data-parallel kernels (section 3); this is an
 * optional monitor, not a step of the path.
 * u_new, u_old: device pointers to the whole domain in one buffer each,
 * shape[0..dims-1] elements (slowest first) of type dtype (CCL_DTYPE_*),
 * element strides pitch[0..dims-2] of the outer dimensions (rows: pitch of
 * the last-but-one dimension >= the row length; 3D planes >= rows x pitch).
 * energy_out: device pointer to one double, written in stream order.  The
 * terms are formed in double from the exactly widened elements and summed
 * in a fixed order (deterministic for a given shape; the summation order is
 * not the oracle's, so the two agree to rounding in double).  The call
 * allocates and frees a small workspace in stream order.
 * Errors: INVALID (NULL, dims, dtype, shape < 1, pitches), HIP. */
ccl_status ccl_wave_energy(int32_t dims, const int64_t *shape, const int64_t *pitch,
                           int32_t dtype, double r2, const void *u_new, const void *u_old,
                           double *energy_out, void *hip_stream);

/* ---- Batched grids ------------------------------------------------------
 * Many independent 2D grids (each its own domain, Dirichlet zero outside)
 * advanced by one persistent kernel launch, captured once in a HIP graph so
 * that a run is a single graph launch.  Each grid uses the same per-cell
 * expression as ccl_wave_step, so its result is bitwise equal to stepping
 * it alone. */
typedef struct {
  int64_t ny, nx;          /* rows, columns                                 */
  int64_t pitch;           /* elements between rows: >= nx, multiple of 4   */
  int32_t steps;           /* leapfrog steps to take, >= 0                  */
  int32_t temporal_depth;  /* T in 1..8 steps per pass over the grid        */
  int32_t tile_rows;       /* rows per tile, >= T; 0 = automatic           */
  float r2;                /* (c dt / dx)^2                                 */
  float *buf[4];           /* device buffers of ny*pitch floats, 16-byte
                              aligned: buf[0] = u^{-1}, buf[1] = u^0 on
                              entry; buf[2], buf[3] are the second pair     */
} ccl_batch_grid;

typedef struct ccl_batch ccl_batch;  /* opaque */

#define CCL_BATCH_NO_GRAPH 1  /* ccl_batch_run launches kernels directly */
#define CCL_BATCH_PER_GRID 2  /* step each grid by its own ccl_wave_step
                                 sequence (one chunk, its own T and tile
                                 rows), grid after grid, instead of the
                                 persistent kernel: each grid's buffers stay
                                 in the last-level cache across its blocks */

/* Plans a batch: tile tables, progress counters and the captured graph
 * (library-owned device memory, released by ccl_batch_destroy).  The grid
 * buffers stay caller-owned and must outlive the batch.
 * Errors: INVALID, RANGE, NOMEM, HIP. */
ccl_status ccl_batch_create(int32_t ngrids, const ccl_batch_grid *grids, int32_t flags,
                            ccl_batch **out);
/* Enqueues one run on `hip_stream`: every grid advances its `steps` from
 * buf[0], buf[1]; a run always starts from that pair.  Errors: INVALID, HIP. */
ccl_status ccl_batch_run(ccl_batch *b, void *hip_stream);
/* Synchronises `hip_stream` and reports TIMEOUT if, during the last run, a
 * tile's wait for its neighbours passed the wait limit (its results are then
 * incomplete).  Errors: INVALID, HIP, TIMEOUT. */
ccl_status ccl_batch_check(ccl_batch *b, void *hip_stream);
/* Wait limit of the dependency waits, in microseconds (default 10 s). */
ccl_status ccl_batch_set_wait_limit(ccl_batch *b, int64_t microseconds);
/* Which buffers hold u^{steps-1} and u^{steps} of `grid` after a run. */
ccl_status ccl_batch_result(const ccl_batch *b, int32_t grid, int32_t *prev_buf,
                            int32_t *cur_buf);
ccl_status ccl_batch_destroy(ccl_batch *b);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one run
 * of the persistent batched kernel, planned on every call: the same kernel
 * and the same results as ccl_batch_create (flags 0 or CCL_BATCH_NO_GRAPH)
 * followed by ccl_batch_run, enqueued on `hip_stream`.  Its tile tables,
 * per-tile progress counters and control words live in a fixed device array
 * of CCL_BATCH_STATIC_BYTES inside the library; every device the library
 * runs on holds its own copy until the process ends.  The call allocates no
 * device memory (no hipMalloc, hipFree or allocating library routine; its
 * host-side plan uses ordinary host memory) and copies the tables host to
 * device on `hip_stream`, then clears the counters with a kernel.
 * Every call on one device shares that device's array, which keeps the last
 * call's contents: calls that overlap on one device (two streams, two host
 * threads) race and must be serialised by the caller.
 *   grids        : as for ccl_batch_create; the buffers are the caller's
 *   prev_buf,
 *   cur_buf      : host arrays of ngrids entries, or NULL: which of each
 *                  grid's buffers hold u^{steps-1} and u^{steps} afterwards
 *   wait_failed  : NULL (the call returns once the work is enqueued) or a
 *                  host int: the call then synchronises `hip_stream` and sets
 *                  it to 1 if a tile's dependency wait passed its 10 s limit
 *                  (results incomplete, status TIMEOUT), else 0
 * Errors: INVALID (as ccl_batch_create), RANGE (the plan needs more than
 * CCL_BATCH_STATIC_BYTES: fewer grids or taller tiles fit), HIP, TIMEOUT. */
#define CCL_BATCH_STATIC_BYTES (4u << 20)
ccl_status ccl_batch_run_static(int32_t ngrids, const ccl_batch_grid *grids,
                                int32_t *prev_buf, int32_t *cur_buf, int32_t *wait_failed,
                                void *hip_stream);

/* ---- Autotuner ------------------------------------------------------------
 * A launch configuration of ccl_wave_step for one domain shape (offset 0,
 * split along dimension 0), and what measuring it gave. */
typedef struct {
  int32_t dims;             /* 2 or 3                                        */
  int64_t shape[3];         /* domain extents, dimension 0 slowest           */
  int32_t nchunks;          /* K device-local chunks                         */
  int32_t temporal_depth;   /* T                                             */
  int32_t tile_rows;        /* rows (2D) / planes (3D) per tile, 0 = auto    */
} ccl_tune_config;

typedef struct {
  double seconds_per_step;  /* median over the timed runs                    */
  double joules_per_step;   /* device energy per step, NaN if not measured   */
  double window_seconds;    /* counter time between the two energy reads     */
  int32_t runs_in_window;
} ccl_tune_sample;

/* Measures each config: ccl_wave_step over zero-filled scratch buffers
 * (allocated for the call and freed before it returns), one warm-up run of
 * `steps` steps, `reps` timed runs (median kept), and — when
 * energy_window_s > 0 and device energy is readable — back-to-back runs
 * until two updates of the device energy counter at least that many seconds
 * apart (by the counter's timestamps) have been seen: joules_per_step is the
 * mean power between them times seconds_per_step.
 * Synchronises `hip_stream`.  Errors: INVALID, RANGE, UNSUPPORTED, HIP. */
ccl_status ccl_autotune_measure(int32_t n, const ccl_tune_config *cfgs, float r2,
                                int32_t steps, int32_t reps, double energy_window_s,
                                int32_t device, void *hip_stream, ccl_tune_sample *out);

/* The autotuner's candidate set for a shape (dims 2 or 3, extents shape[0..
 * dims-1]): K device-local chunks in {1, 2, 4, 8, 16} (at most shape[0]),
 * tile rows / planes in {0 = automatic, 16, 32, 64, 128} and T in 1..8, in
 * that nesting order (K slowest); only K == nchunks when nchunks > 0.
 * Writes min(count, max_out) configs to out (host) and the count to *n_out.
 * Host only.  Errors: INVALID, RANGE (count > max_out; *n_out still set). */
ccl_status ccl_autotune_candidates(int32_t dims, const int64_t *shape, int32_t nchunks,
                                   int32_t max_out, ccl_tune_config *out, int32_t *n_out);

/* Objectives of a sweep: time per step, energy per step, their product. */
#define CCL_OBJECTIVE_TIME 0
#define CCL_OBJECTIVE_ENERGY 1
#define CCL_OBJECTIVE_EDP 2

/* The exhaustive sweep of the paper's per-kernel tuning (section 4: picking
 * a launch configuration per kernel by a target metric): every candidate of
 * ccl_autotune_candidates measured by ccl_autotune_measure (with the same
 * r2, steps, reps, energy window, device and stream), the configs and
 * samples written to cfgs_out / out (host, room for max_out), their count
 * to *n_out, and to *best the index of the smallest measured objective
 * (CCL_OBJECTIVE_*; ties: the lowest index).  Energy objectives need
 * energy_window_s > 0.  Synchronises the stream.
 * Errors: INVALID, RANGE, UNSUPPORTED (no energy read), HIP. */
ccl_status ccl_autotune_sweep(int32_t dims, const int64_t *shape, int32_t nchunks, float r2,
                              int32_t steps, int32_t reps, double energy_window_s,
                              int32_t objective, int32_t device, void *hip_stream,
                              int32_t max_out, ccl_tune_config *cfgs_out, ccl_tune_sample *out,
                              int32_t *n_out, int32_t *best);

/* Rows (2D) / planes (3D) per tile that ccl_wave_step uses for `c` when its
 * tile_rows is 0: the value minimising (resident-wave rounds) x (rows + 2
 * halo rows) for the device's occupancy of the depth-T kernel; tile_rows
 * itself when it is positive.  Errors: INVALID, RANGE. */
ccl_status ccl_wave_plan_rows(const ccl_tune_config *c, int32_t *rows);

/* Waves of the stencil kernel for (dims, T) that the current device holds
 * at once, as the occupancy API reports them (the figure the row planner
 * uses; a fixed guess where no device answers).  Errors: INVALID. */
ccl_status ccl_wave_slots(int32_t dims, int32_t T, int64_t *slots);

/* Cost-model features of each config (host array n x CCL_MLP_IN), from the
 * launch geometry the kernels would use (rows as ccl_wave_plan_rows gives
 * them, chunks as ccl_split_range cuts dim 0):
 *   0-2  log2 of the three extents (0 for the third in 2D)
 *   3    1 for 3D, 0 for 2D
 *   4    log2 of the redundancy: cells the waves stream per launch (tile
 *        overlap included) / cells of the domain
 *   5    log2 K          6  log2 tile rows          7  T
 *   8    last-round fill: waves / (ceil(waves / slots) * slots), slots from
 *        ccl_wave_slots
 *   9    log2(1 + halo bytes per step)
 *   10   modelled HBM bytes per cell-step (12 for T = 1, 16/T otherwise)
 *   11   log2 waves per launch
 * Errors: INVALID, RANGE (more chunks than rows). */
ccl_status ccl_costmodel_features(int32_t n, const ccl_tune_config *cfgs, float *x_host);

/* ---- Launch-config cost model ------------------------------------------
 * A 12-64-64-2 float32 MLP (ReLU hidden layers) that maps the features of a
 * launch config to two predicted targets (the library's tuner uses [log time
 * per cell-step, log device power], standardised by the caller; the kernels
 * do not depend on what the targets mean).  Trained on the GPU by the library's own
 * forward/backward kernels with L = 1/(2n) sum w |y - t|^2 and Adam; gradients
 * are summed in a fixed order, so training is deterministic.  Parameters are
 * packed W1 (64x12), b1 (64), W2 (64x64), b2 (64), W3 (2x64), b3 (2),
 * row-major W[out][in].  All sample arrays are device memory, row-major
 * n x 12 (x) and n x 2 (t, y). */
#define CCL_MLP_IN 12
#define CCL_MLP_HIDDEN 64
#define CCL_MLP_OUT 2
#define CCL_MLP_NPARAMS 5122
enum { CCL_MLP_PARAMS = 0, CCL_MLP_GRADS = 1, CCL_MLP_LOSS = 2 };
typedef struct ccl_mlp ccl_mlp;  /* opaque: parameters, gradient, Adam state */

/* Copies CCL_MLP_NPARAMS host floats into a new model.
 * Errors: INVALID (NULL, non-finite), HIP. */
ccl_status ccl_mlp_create(const float *params, ccl_mlp **out);
ccl_status ccl_mlp_destroy(ccl_mlp *m);
/* Copies parameters, the last gradient, or the last loss (1 float) to host. */
ccl_status ccl_mlp_get(const ccl_mlp *m, int32_t what, float *host_out);
/* y = net(x) for n samples. */
ccl_status ccl_mlp_forward(ccl_mlp *m, int32_t n, const float *x, float *y, void *hip_stream);
/* Gradient and loss of L over the n samples (x, t), kept in the model. */
ccl_status ccl_mlp_grad(ccl_mlp *m, int32_t n, const float *x, const float *t,
                        void *hip_stream);
/* The same with per-output sample weights w (device, n x 2, may be NULL):
 * L = 1/(2n) sum w_bk (y_bk - t_bk)^2; a zero weight masks a missing label. */
ccl_status ccl_mlp_grad_weighted(ccl_mlp *m, int32_t n, const float *x, const float *t,
                                 const float *w, void *hip_stream);
/* One Adam step with the kept gradient (bias-corrected; step count kept). */
ccl_status ccl_mlp_adam(ccl_mlp *m, float lr, float beta1, float beta2, float eps,
                        void *hip_stream);
/* `epochs` full-batch steps of weighted grad + Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8); w may be NULL. */
ccl_status ccl_mlp_train(ccl_mlp *m, int32_t n, const float *x, const float *t,
                         const float *w, int32_t epochs, float lr, void *hip_stream);
/* Scores score_i = w_time*y_i0 + w_energy*y_i1 of n candidates and writes the
 * index of the smallest (ties: lowest index) to *best (device int32);
 * `scores` (device, n floats) may be NULL. */
ccl_status ccl_mlp_pick(ccl_mlp *m, int32_t n, const float *x, float w_time, float w_energy,
                        float *scores, int32_t *best, void *hip_stream);

/* The k candidates with the smallest scores score_i = w_time*y_i0 +
 * w_energy*y_i1 (the same scores as ccl_mlp_pick), in ascending order of
 * score (ties: lower index first), as indices into x's n rows written to
 * order (device int32, k entries); order[0] is ccl_mlp_pick's choice.
 * 1 <= k <= n <= 4096 (one block holds every score in LDS).
 * Errors: INVALID, RANGE, HIP. */
ccl_status ccl_mlp_rank(ccl_mlp *m, int32_t n, const float *x, float w_time, float w_energy,
                        int32_t k, int32_t *order, void *hip_stream);

/* Kernel launch timing, for measurement.  While enabled, every launch of
 * the kernel families below is bracketed by HIP events recorded on the
 * stream it is launched on.  ccl_timing_enable(on) discards earlier records
 * and switches recording on or off; ccl_timing_query waits for the recorded
 * events of one family and returns their count and summed duration (ms).
 * Errors: INVALID, HIP. */
enum {
  CCL_KERNEL_STENCIL = 0,  /* the wave-stencil kernels (2D, 3D, batched)    */
  CCL_KERNEL_HALO = 1,     /* halo exchange / pack / unpack copies          */
  CCL_KERNEL_SAXPY = 2,
  CCL_KERNEL_BATCH = 3,    /* whole batched runs (one graph launch each)    */
  CCL_KERNEL_KINDS = 4
};
ccl_status ccl_timing_enable(int32_t on);
ccl_status ccl_timing_query(int32_t kernel, int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif

#endif /* CCL_H */
