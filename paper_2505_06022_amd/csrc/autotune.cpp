// Autotuner: measures launch configurations of the chunked stencil and
// encodes configs as cost-model features.
//
// A measurement runs the real entry point (ccl_wave_step, halo exchanges
// included) on zero-filled scratch buffers of the candidate's shape, split
// into its chunk count with regions sized by NEIGHBORHOOD(T): one warm-up
// run, then `reps` timed runs (HIP events on the caller's stream; the median
// is kept), then, if asked, repeated runs inside a window of at least
// `energy_window_s` seconds bracketed by device-energy reads.  The scratch
// pool is library-owned for the duration of the call.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "ccl_internal.h"

namespace ccl {
namespace {

struct Plan {
  std::vector<ccl_chunk> chunks;
  std::vector<ccl_subrange> regions;
  std::vector<int64_t> elems;   // per buffer
  int nbuf = 2;
  size_t bytes = 0;
};

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

ccl_status plan_of(const ccl_tune_config &c, Plan *P) {
  const int dims = c.dims;
  if (dims != 2 && dims != 3) return fail(CCL_E_INVALID, "dims=%d must be 2 or 3", dims);
  if (c.temporal_depth < 1 || c.temporal_depth > CCL_MAX_DEPTH)
    return fail(CCL_E_INVALID, "temporal depth %d", c.temporal_depth);
  ccl_subrange r;
  memset(&r, 0, sizeof(r));
  r.dims = dims;
  for (int d = 0; d < dims; ++d) r.range[d] = c.shape[d];
  P->chunks.resize(std::max(1, c.nchunks));
  ccl_status st = ccl_split_range(&r, c.nchunks, 0, P->chunks.data());
  if (st != CCL_OK) return st;
  ccl_range_mapper m;
  memset(&m, 0, sizeof(m));
  m.kind = CCL_MAP_NEIGHBORHOOD;
  for (int d = 0; d < dims; ++d) m.extent[d] = c.temporal_depth;
  P->nbuf = c.temporal_depth > 1 ? 4 : 2;
  P->regions.resize(c.nchunks);
  P->elems.resize(c.nchunks);
  P->bytes = 0;
  for (int k = 0; k < c.nchunks; ++k) {
    st = ccl_region_of(&P->chunks[k], &m, c.shape, &P->regions[k]);
    if (st != CCL_OK) return st;
    int64_t e = round_up(P->regions[k].range[dims - 1], 64);
    for (int d = 0; d + 1 < dims; ++d) e *= P->regions[k].range[d];
    P->elems[k] = e;
    P->bytes += static_cast<size_t>(round_up(e * 4, 256)) * P->nbuf;
  }
  return CCL_OK;
}

}  // namespace
}  // namespace ccl

using namespace ccl;

extern "C" ccl_status ccl_autotune_measure(int32_t n, const ccl_tune_config *cfgs, float r2,
                                           int32_t steps, int32_t reps,
                                           double energy_window_s, int32_t device,
                                           void *hip_stream, ccl_tune_sample *out) {
  clear_error();
  if (n < 0 || (n > 0 && (!cfgs || !out))) return fail(CCL_E_INVALID, "bad arguments");
  if (steps < 1 || reps < 1) return fail(CCL_E_INVALID, "steps and reps must be >= 1");
  if (!std::isfinite(r2) || r2 < 0.0f) return fail(CCL_E_INVALID, "bad r2");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  std::vector<Plan> plans(n);
  size_t pool_bytes = 0;
  for (int i = 0; i < n; ++i) {
    ccl_status st = plan_of(cfgs[i], &plans[i]);
    if (st != CCL_OK) return fail(st, "config %d: %s", i, ccl_last_error());
    pool_bytes = std::max(pool_bytes, plans[i].bytes);
  }
  void *pool = nullptr;
  ccl_status st = hip_check(hipMalloc(&pool, std::max<size_t>(pool_bytes, 256)),
                            "hipMalloc(autotune pool)");
  if (st != CCL_OK) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  st = hip_check(hipEventCreate(&e0), "hipEventCreate");
  if (st == CCL_OK) st = hip_check(hipEventCreate(&e1), "hipEventCreate");
  const bool want_energy = energy_window_s > 0.0;
  for (int i = 0; i < n && st == CCL_OK; ++i) {
    const ccl_tune_config &c = cfgs[i];
    Plan &P = plans[i];
    const int dims = c.dims;
    st = hip_check(hipMemsetAsync(pool, 0, P.bytes, s), "hipMemsetAsync");
    if (st != CCL_OK) break;
    std::vector<ccl_chunk_buffer> bufs(4 * c.nchunks);
    char *cursor = static_cast<char *>(pool);
    for (int b = 0; b < P.nbuf; ++b)
      for (int k = 0; k < c.nchunks; ++k) {
        ccl_chunk_buffer &B = bufs[b * c.nchunks + k];
        memset(&B, 0, sizeof(B));
        B.base = cursor;
        B.region = P.regions[k];
        const int64_t row = round_up(P.regions[k].range[dims - 1], 64);
        B.pitch[dims - 1] = 1;
        B.pitch[dims - 2] = row;
        if (dims == 3) B.pitch[0] = row * P.regions[k].range[1];
        cursor += round_up(P.elems[k] * 4, 256);
      }
    ccl_chunk_buffer *up = &bufs[0], *uc = &bufs[c.nchunks];
    ccl_chunk_buffer *wp = P.nbuf == 4 ? &bufs[2 * c.nchunks] : nullptr;
    ccl_chunk_buffer *wc = P.nbuf == 4 ? &bufs[3 * c.nchunks] : nullptr;
    ccl_wave_params wp_params;
    memset(&wp_params, 0, sizeof(wp_params));
    wp_params.dims = dims;
    wp_params.r2 = r2;
    wp_params.temporal_depth = c.temporal_depth;
    wp_params.tile_rows = c.tile_rows;
    auto run = [&]() {
      return ccl_wave_step(&wp_params, c.nchunks, P.chunks.data(), up, uc, wp, wc, steps, s);
    };
    st = run();  // warm-up
    if (st != CCL_OK) break;
    std::vector<float> times;
    for (int r = 0; r < reps && st == CCL_OK; ++r) {
      st = hip_check(hipEventRecord(e0, s), "hipEventRecord");
      if (st == CCL_OK) st = run();
      if (st == CCL_OK) st = hip_check(hipEventRecord(e1, s), "hipEventRecord");
      if (st == CCL_OK) st = hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
      float ms = 0.0f;
      if (st == CCL_OK) st = hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
      times.push_back(ms);
    }
    if (st != CCL_OK) break;
    std::sort(times.begin(), times.end());
    const double med_s = 1e-3 * times[times.size() / 2];
    ccl_tune_sample &o = out[i];
    o.seconds_per_step = med_s / steps;
    o.joules_per_step = std::numeric_limits<double>::quiet_NaN();
    o.window_seconds = 0.0;
    o.runs_in_window = 0;
    if (want_energy) {
      // The device counter advances in coarse steps (about once a second on
      // the MI355X boxes): run back to back and take the energy between two
      // counter updates (changes of its value) at least energy_window_s
      // apart by the counter's own timestamps; J/step = mean power x the
      // timed seconds per step.  A counter that goes back restarts the window.
      double j = 0.0, prev = 0.0, ja = 0.0;
      uint64_t ts = 0, tsa = 0;
      bool have_a = false, done = false;
      int runs = 0;
      const auto t0 = std::chrono::steady_clock::now();
      if (ccl_energy_read(device, s, &prev, &ts) == CCL_OK) {
        while (!done) {
          st = run();
          if (st != CCL_OK) break;
          ++runs;
          if (ccl_energy_read(device, s, &j, &ts) != CCL_OK) break;
          if (j != prev) {
            if (!have_a || j < ja || ts <= tsa) {
              have_a = true;
              ja = j;
              tsa = ts;
              runs = 0;
            } else if (static_cast<double>(ts - tsa) * 1e-9 >= energy_window_s) {
              const double watts = (j - ja) / (static_cast<double>(ts - tsa) * 1e-9);
              if (watts > 0.0 && std::isfinite(watts)) {
                o.joules_per_step = watts * o.seconds_per_step;
                o.window_seconds = static_cast<double>(ts - tsa) * 1e-9;
                o.runs_in_window = runs;
              }
              done = true;
            }
          }
          prev = j;
          const double el =
              std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
          if (el > 10.0 * energy_window_s + 5.0) break;  // counter not advancing
        }
      }
      if (st != CCL_OK) break;
      clear_error();
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  (void)hipFree(pool);
  return st;
}

// The library's candidate set for a shape: K in {1, 2, 4, 8, 16} (at most
// the extent along dimension 0), tile rows / planes in {0 (automatic), 16,
// 32, 64, 128}, T in 1..8, in that nesting order (K slowest).
static const int32_t kCandK[] = {1, 2, 4, 8, 16};
static const int32_t kCandRows[] = {0, 16, 32, 64, 128};

extern "C" ccl_status ccl_autotune_candidates(int32_t dims, const int64_t *shape, int32_t nchunks,
                                              int32_t max_out, ccl_tune_config *out,
                                              int32_t *n_out) {
  clear_error();
  if ((dims != 2 && dims != 3) || !shape || !n_out || max_out < 0 || (max_out > 0 && !out))
    return fail(CCL_E_INVALID, "bad arguments");
  for (int d = 0; d < dims; ++d)
    if (shape[d] < 1) return fail(CCL_E_INVALID, "empty extent");
  int32_t n = 0;
  for (int32_t K : kCandK) {
    if (K > shape[0] || (nchunks > 0 && K != nchunks)) continue;
    for (int32_t rows : kCandRows)
      for (int32_t T = 1; T <= CCL_MAX_DEPTH; ++T) {
        if (n < max_out) {
          ccl_tune_config &c = out[n];
          memset(&c, 0, sizeof(c));
          c.dims = dims;
          for (int d = 0; d < dims; ++d) c.shape[d] = shape[d];
          c.nchunks = K;
          c.temporal_depth = T;
          c.tile_rows = rows;
        }
        ++n;
      }
  }
  *n_out = n;
  if (n > max_out) return fail(CCL_E_RANGE, "%d candidates, room for %d", n, max_out);
  return CCL_OK;
}

extern "C" ccl_status ccl_autotune_sweep(int32_t dims, const int64_t *shape, int32_t nchunks,
                                         float r2, int32_t steps, int32_t reps,
                                         double energy_window_s, int32_t objective,
                                         int32_t device, void *hip_stream, int32_t max_out,
                                         ccl_tune_config *cfgs_out, ccl_tune_sample *out,
                                         int32_t *n_out, int32_t *best) {
  clear_error();
  if (!best || !out) return fail(CCL_E_INVALID, "NULL argument");
  if (objective < CCL_OBJECTIVE_TIME || objective > CCL_OBJECTIVE_EDP)
    return fail(CCL_E_INVALID, "objective %d", objective);
  if (objective != CCL_OBJECTIVE_TIME && !(energy_window_s > 0.0))
    return fail(CCL_E_INVALID, "an energy objective needs energy_window_s > 0");
  ccl_status st = ccl_autotune_candidates(dims, shape, nchunks, max_out, cfgs_out, n_out);
  if (st != CCL_OK) return st;
  const int32_t n = *n_out;
  if (n == 0) return fail(CCL_E_RANGE, "no candidate has %d chunks", nchunks);
  st = ccl_autotune_measure(n, cfgs_out, r2, steps, reps, energy_window_s, device, hip_stream,
                            out);
  if (st != CCL_OK) return st;
  // the smallest measured objective; ties and unmeasured energies: the
  // lower index is kept
  int32_t b = -1;
  double bv = std::numeric_limits<double>::infinity();
  for (int32_t i = 0; i < n; ++i) {
    const double t = out[i].seconds_per_step, j = out[i].joules_per_step;
    const double v = objective == CCL_OBJECTIVE_TIME     ? t
                     : objective == CCL_OBJECTIVE_ENERGY ? j
                                                         : t * j;
    if (std::isfinite(v) && v < bv) {
      bv = v;
      b = i;
    }
  }
  if (b < 0) return fail(CCL_E_UNSUPPORTED, "no candidate was measured for this objective");
  *best = b;
  return CCL_OK;
}

extern "C" ccl_status ccl_wave_plan_rows(const ccl_tune_config *c, int32_t *rows) {
  clear_error();
  if (!c || !rows) return fail(CCL_E_INVALID, "NULL argument");
  if ((c->dims != 2 && c->dims != 3) || c->nchunks < 1 || c->temporal_depth < 1 ||
      c->temporal_depth > CCL_MAX_DEPTH)
    return fail(CCL_E_INVALID, "malformed config");
  for (int d = 0; d < c->dims; ++d)
    if (c->shape[d] < 1) return fail(CCL_E_INVALID, "empty extent");
  if (c->nchunks > c->shape[0]) return fail(CCL_E_RANGE, "more chunks than rows");
  if (c->tile_rows > 0) {
    *rows = c->tile_rows;
    return CCL_OK;
  }
  *rows = c->dims == 2
              ? wave2d_plan_rows(c->shape[0], c->shape[1], c->nchunks, c->temporal_depth)
              : wave3d_plan_planes(c->shape[0], c->shape[1], c->shape[2], c->nchunks,
                                   c->temporal_depth);
  return CCL_OK;
}

extern "C" ccl_status ccl_wave_slots(int32_t dims, int32_t T, int64_t *slots) {
  clear_error();
  if (!slots) return fail(CCL_E_INVALID, "NULL argument");
  if ((dims != 2 && dims != 3) || T < 1 || T > CCL_MAX_DEPTH)
    return fail(CCL_E_INVALID, "dims=%d, T=%d", dims, T);
  *slots = dims == 2 ? wave2d_slots(T) : wave3d_slots(T);
  return CCL_OK;
}

namespace ccl {
namespace {

// Launch geometry of one config as the kernels tile it: waves per launch
// and the cells the waves stream (overlap included) per useful cell.
struct Geometry {
  double waves = 0.0;
  double redundancy = 1.0;
};

Geometry geometry_of(const ccl_tune_config &c, int32_t rows) {
  const int T = c.temporal_depth, K = c.nchunks;
  const int64_t n0 = c.shape[0], n1 = c.shape[1], n2 = c.dims == 3 ? c.shape[2] : 1;
  const int A = 4 * ((T + 3) / 4);
  double waves = 0.0, streamed = 0.0;
  for (int k = 0; k < K; ++k) {
    const int64_t nk = (k + 1) * n0 / K - k * n0 / K;  // the split of ccl_split_range
    const int64_t segs = (nk + rows - 1) / rows;
    if (c.dims == 2) {
      const int64_t strips = (n1 + (256 - 2 * A) - 1) / (256 - 2 * A);
      waves += static_cast<double>(segs * strips);
      streamed += static_cast<double>(segs) * (rows + 2.0 * T) * strips * 256.0;
    } else if (T == 1) {
      const int64_t strips = (n2 + 255) / 256, rowblk = (n1 + 3) / 4;
      waves += static_cast<double>(segs * strips * rowblk);
      // each wave also loads the two rows around its four
      streamed += static_cast<double>(segs) * (rows + 2.0) * strips * 256.0 * rowblk * 6.0;
    } else {
      int32_t oc = 1, orows = 1, wpb = 1;
      wave3d_tb_geometry(T, &oc, &orows, &wpb);
      const int64_t strips = (n2 + oc - 1) / oc, rowblk = (n1 + orows - 1) / orows;
      waves += static_cast<double>(segs * strips * rowblk * wpb);
      streamed += static_cast<double>(segs) * (rows + 2.0 * T) * strips * (oc + 2.0 * A) *
                  rowblk * (orows + 2.0 * T);
    }
  }
  Geometry g;
  g.waves = waves;
  g.redundancy = streamed / (static_cast<double>(n0) * n1 * n2);
  return g;
}

}  // namespace
}  // namespace ccl

extern "C" ccl_status ccl_costmodel_features(int32_t n, const ccl_tune_config *cfgs,
                                             float *x_host) {
  clear_error();
  if (n < 0 || (n > 0 && (!cfgs || !x_host))) return fail(CCL_E_INVALID, "bad arguments");
  for (int i = 0; i < n; ++i) {
    const ccl_tune_config &c = cfgs[i];
    if ((c.dims != 2 && c.dims != 3) || c.nchunks < 1 || c.temporal_depth < 1 ||
        c.temporal_depth > CCL_MAX_DEPTH || c.tile_rows < 0)
      return fail(CCL_E_INVALID, "config %d is malformed", i);
    for (int d = 0; d < c.dims; ++d)
      if (c.shape[d] < 1) return fail(CCL_E_INVALID, "config %d has an empty extent", i);
    if (c.nchunks > c.shape[0]) return fail(CCL_E_RANGE, "config %d: more chunks than rows", i);
    const double n0 = static_cast<double>(c.shape[0]);
    const double n1 = static_cast<double>(c.shape[1]);
    const double n2 = c.dims == 3 ? static_cast<double>(c.shape[2]) : 1.0;
    const double T = c.temporal_depth;
    const double K = c.nchunks;
    int32_t rows = 0;
    if (ccl_wave_plan_rows(&c, &rows) != CCL_OK)
      return fail(CCL_E_INVALID, "config %d: %s", i, ccl_last_error());
    const Geometry g = geometry_of(c, rows);
    const double slots = static_cast<double>(
        c.dims == 2 ? wave2d_slots(c.temporal_depth) : wave3d_slots(c.temporal_depth));
    const double rounds = std::ceil(g.waves / slots);
    // halo bytes per step: 2 directions x (K-1) boundaries x (2T-1) rows/planes
    // of u^n and u^{n-1}, read and written, per T steps
    const double row_bytes = 4.0 * n1 * n2;
    const double halo = 2.0 * (K - 1.0) * (2.0 * T - 1.0) * row_bytes * 2.0 / T;
    const double model_bytes = c.temporal_depth == 1 ? 12.0 : 16.0 / T;
    float *x = x_host + static_cast<size_t>(i) * CCL_MLP_IN;
    x[0] = static_cast<float>(std::log2(n0));
    x[1] = static_cast<float>(std::log2(n1));
    x[2] = static_cast<float>(c.dims == 3 ? std::log2(n2) : 0.0);
    x[3] = c.dims == 3 ? 1.0f : 0.0f;
    x[4] = static_cast<float>(std::log2(g.redundancy));
    x[5] = static_cast<float>(std::log2(K));
    x[6] = static_cast<float>(std::log2(static_cast<double>(rows)));
    x[7] = static_cast<float>(T);
    x[8] = static_cast<float>(g.waves / (rounds * slots));
    x[9] = static_cast<float>(std::log2(1.0 + halo));
    x[10] = static_cast<float>(model_bytes);
    x[11] = static_cast<float>(std::log2(std::max(1.0, g.waves)));
  }
  return CCL_OK;
}
