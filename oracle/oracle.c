/*
 * CPU oracle for the chunked leapfrog wave stencil.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header or constant with the HIP
 * path.
 *
 * What it computes (plain definition, no blocking, fusion or reordering):
 *
 *   Grid: D in {1,2,3}, every cell of the n_0 x ... x n_{D-1} box is an
 *   unknown; a ghost layer one cell wide around the box holds zeros
 *   (homogeneous Dirichlet).  The ghost layer is stored explicitly here, so
 *   the update loop reads every neighbour from the padded array.
 *
 *   Second-order central-difference leapfrog for u_tt = c^2 lap(u) with
 *   r^2 = (c dt / dx)^2, in one canonical evaluation order:
 *     2D: s = (u[i-1][j] + u[i+1][j]) + (u[i][j-1] + u[i][j+1])
 *         lap = s - 4 u[i][j]
 *     3D: s = ((u[z-1] + u[z+1]) + (u[y-1] + u[y+1])) + (u[x-1] + u[x+1])
 *         lap = s - 6 u
 *     1D: s = u[i-1] + u[i+1], lap = s - 2 u
 *     u_next = fma(r^2, lap, 2 u - u_prev)
 *   The same expression is applied in float and in double.  Compiled with
 *   -ffp-contract=off so that the only fused operation is the written fma.
 *
 *   Discrete energy (an invariant of the scheme, see oracle_energy*):
 *     E^{n+1/2} = sum_i (u^{n+1}_i - u^n_i)^2
 *               + r^2 sum_{edges (a,b)} (u^{n+1}_a - u^{n+1}_b)(u^n_a - u^n_b)
 *   over all edges of the padded grid (edges to the zero ghosts included).
 *
 *   SAXPY: z_i = fma(a, x_i, y_i) in float, the data-parallel kernel of the
 *   paper's first listing (section 2), used to calibrate bandwidth.
 *
 *   16-bit storage (oracle_wave_stored): the fields kept in bfloat16 or
 *   binary16 between passes of `depth` float steps, rounded to nearest
 *   even when stored (oracle_round_to_format).
 *
 * Parallelism: an optional OpenMP loop over the slowest axis; each cell's
 * arithmetic is unchanged by it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL -1
#define ORACLE_ENOMEM -5

/* ------------------------------------------------------------------ 2D -- */

/* Padded index: cell (i, j), i in [-1, ny], j in [-1, nx]. */
#define P2(i, j) ((size_t)((i) + 1) * (size_t)(nx + 2) + (size_t)((j) + 1))

#define WAVE2D_BODY(T, FMA, FOUR, TWO)                                         \
  if (ny < 1 || nx < 1 || steps < 0 || !u_prev0 || !u_cur0 || !u_prev_out ||    \
      !u_cur_out)                                                              \
    return ORACLE_EINVAL;                                                      \
  size_t npad = (size_t)(ny + 2) * (size_t)(nx + 2);                           \
  T *prev = (T *)calloc(npad, sizeof(T));                                      \
  T *cur = (T *)calloc(npad, sizeof(T));                                       \
  T *next = (T *)calloc(npad, sizeof(T));                                      \
  if (!prev || !cur || !next) {                                                \
    free(prev); free(cur); free(next);                                         \
    return ORACLE_ENOMEM;                                                      \
  }                                                                            \
  for (int64_t i = 0; i < ny; ++i)                                             \
    for (int64_t j = 0; j < nx; ++j) {                                         \
      prev[P2(i, j)] = u_prev0[i * nx + j];                                    \
      cur[P2(i, j)] = u_cur0[i * nx + j];                                      \
    }                                                                          \
  for (int64_t s = 0; s < steps; ++s) {                                        \
    _Pragma("omp parallel for num_threads(threads) schedule(static)")          \
    for (int64_t i = 0; i < ny; ++i)                                           \
      for (int64_t j = 0; j < nx; ++j) {                                       \
        T c = cur[P2(i, j)];                                                   \
        T sum = (cur[P2(i - 1, j)] + cur[P2(i + 1, j)]) +                      \
                (cur[P2(i, j - 1)] + cur[P2(i, j + 1)]);                       \
        T lap = sum - FOUR * c;                                                \
        next[P2(i, j)] = FMA(r2, lap, TWO * c - prev[P2(i, j)]);               \
      }                                                                        \
    T *t = prev; prev = cur; cur = next; next = t;                             \
  }                                                                            \
  for (int64_t i = 0; i < ny; ++i)                                             \
    for (int64_t j = 0; j < nx; ++j) {                                         \
      u_prev_out[i * nx + j] = prev[P2(i, j)];                                 \
      u_cur_out[i * nx + j] = cur[P2(i, j)];                                   \
    }                                                                          \
  free(prev); free(cur); free(next);                                           \
  return ORACLE_OK;

/* Advance (u_prev0, u_cur0) = (u^{-1}, u^0) by `steps` leapfrog steps;
 * writes (u^{steps-1}, u^{steps}).  Arrays are ny x nx row-major. */
int oracle_wave2d_f32(int64_t ny, int64_t nx, float r2, int64_t steps,
                      const float *u_prev0, const float *u_cur0,
                      float *u_prev_out, float *u_cur_out, int threads) {
  if (threads < 1) threads = 1;
  WAVE2D_BODY(float, fmaf, 4.0f, 2.0f)
}

int oracle_wave2d_f64(int64_t ny, int64_t nx, double r2, int64_t steps,
                      const double *u_prev0, const double *u_cur0,
                      double *u_prev_out, double *u_cur_out, int threads) {
  if (threads < 1) threads = 1;
  WAVE2D_BODY(double, fma, 4.0, 2.0)
}

/* ------------------------------------------------------------------ 3D -- */

#define P3(z, y, x)                                                            \
  (((size_t)((z) + 1) * (size_t)(ny + 2) + (size_t)((y) + 1)) *                \
       (size_t)(nx + 2) +                                                      \
   (size_t)((x) + 1))

#define WAVE3D_BODY(T, FMA, SIX, TWO)                                          \
  if (nz < 1 || ny < 1 || nx < 1 || steps < 0 || !u_prev0 || !u_cur0 ||         \
      !u_prev_out || !u_cur_out)                                               \
    return ORACLE_EINVAL;                                                      \
  size_t npad = (size_t)(nz + 2) * (size_t)(ny + 2) * (size_t)(nx + 2);        \
  T *prev = (T *)calloc(npad, sizeof(T));                                      \
  T *cur = (T *)calloc(npad, sizeof(T));                                       \
  T *next = (T *)calloc(npad, sizeof(T));                                      \
  if (!prev || !cur || !next) {                                                \
    free(prev); free(cur); free(next);                                         \
    return ORACLE_ENOMEM;                                                      \
  }                                                                            \
  for (int64_t z = 0; z < nz; ++z)                                             \
    for (int64_t y = 0; y < ny; ++y)                                           \
      for (int64_t x = 0; x < nx; ++x) {                                       \
        size_t q = ((size_t)z * (size_t)ny + (size_t)y) * (size_t)nx + (size_t)x; \
        prev[P3(z, y, x)] = u_prev0[q];                                        \
        cur[P3(z, y, x)] = u_cur0[q];                                          \
      }                                                                        \
  for (int64_t s = 0; s < steps; ++s) {                                        \
    _Pragma("omp parallel for num_threads(threads) schedule(static)")          \
    for (int64_t z = 0; z < nz; ++z)                                           \
      for (int64_t y = 0; y < ny; ++y)                                         \
        for (int64_t x = 0; x < nx; ++x) {                                     \
          T c = cur[P3(z, y, x)];                                              \
          T sum = ((cur[P3(z - 1, y, x)] + cur[P3(z + 1, y, x)]) +             \
                   (cur[P3(z, y - 1, x)] + cur[P3(z, y + 1, x)])) +            \
                  (cur[P3(z, y, x - 1)] + cur[P3(z, y, x + 1)]);               \
          T lap = sum - SIX * c;                                               \
          next[P3(z, y, x)] = FMA(r2, lap, TWO * c - prev[P3(z, y, x)]);       \
        }                                                                      \
    T *t = prev; prev = cur; cur = next; next = t;                             \
  }                                                                            \
  for (int64_t z = 0; z < nz; ++z)                                             \
    for (int64_t y = 0; y < ny; ++y)                                           \
      for (int64_t x = 0; x < nx; ++x) {                                       \
        size_t q = ((size_t)z * (size_t)ny + (size_t)y) * (size_t)nx + (size_t)x; \
        u_prev_out[q] = prev[P3(z, y, x)];                                     \
        u_cur_out[q] = cur[P3(z, y, x)];                                       \
      }                                                                        \
  free(prev); free(cur); free(next);                                           \
  return ORACLE_OK;

int oracle_wave3d_f32(int64_t nz, int64_t ny, int64_t nx, float r2, int64_t steps,
                      const float *u_prev0, const float *u_cur0,
                      float *u_prev_out, float *u_cur_out, int threads) {
  if (threads < 1) threads = 1;
  WAVE3D_BODY(float, fmaf, 6.0f, 2.0f)
}

int oracle_wave3d_f64(int64_t nz, int64_t ny, int64_t nx, double r2, int64_t steps,
                      const double *u_prev0, const double *u_cur0,
                      double *u_prev_out, double *u_cur_out, int threads) {
  if (threads < 1) threads = 1;
  WAVE3D_BODY(double, fma, 6.0, 2.0)
}

/* ------------------------------------------------------------------ 1D -- */

int oracle_wave1d_f64(int64_t n, double r2, int64_t steps, const double *u_prev0,
                      const double *u_cur0, double *u_prev_out, double *u_cur_out) {
  if (n < 1 || steps < 0 || !u_prev0 || !u_cur0 || !u_prev_out || !u_cur_out)
    return ORACLE_EINVAL;
  double *prev = (double *)calloc((size_t)n + 2, sizeof(double));
  double *cur = (double *)calloc((size_t)n + 2, sizeof(double));
  double *next = (double *)calloc((size_t)n + 2, sizeof(double));
  if (!prev || !cur || !next) {
    free(prev); free(cur); free(next);
    return ORACLE_ENOMEM;
  }
  for (int64_t i = 0; i < n; ++i) {
    prev[i + 1] = u_prev0[i];
    cur[i + 1] = u_cur0[i];
  }
  for (int64_t s = 0; s < steps; ++s) {
    for (int64_t i = 1; i <= n; ++i) {
      double c = cur[i];
      double lap = (cur[i - 1] + cur[i + 1]) - 2.0 * c;
      next[i] = fma(r2, lap, 2.0 * c - prev[i]);
    }
    double *t = prev; prev = cur; cur = next; next = t;
  }
  for (int64_t i = 0; i < n; ++i) {
    u_prev_out[i] = prev[i + 1];
    u_cur_out[i] = cur[i + 1];
  }
  free(prev); free(cur); free(next);
  return ORACLE_OK;
}

/* ------------------------------------------- 16-bit storage variants -- */

/* Rounding of a float to a narrower binary floating-point format, by the
 * definition of round-to-nearest, ties to even: the representable numbers
 * of a format with `mant` stored fraction bits and smallest normal exponent
 * `emin` are the integer multiples of 2^(e - mant) around 2^e, where
 * e = max(floor(log2 |x|), emin) (below 2^emin the spacing stays
 * 2^(emin - mant): the subnormals).  x / q is exact in double (q is a power
 * of two in range), nearbyint rounds it to an integer with ties to even
 * (the default rounding mode), and anything above the largest finite value
 * `maxfin` after rounding is an infinity.
 *   bfloat16: mant 7, emin -126, maxfin (2 - 2^-7) 2^127
 *   binary16: mant 10, emin -14, maxfin 65504 */
static float round_narrow(float x, int mant, int emin, double maxfin) {
  if (x == 0.0f || !isfinite(x)) return x;
  int ex;
  (void)frexp((double)x, &ex); /* |x| = m 2^ex, m in [1/2, 1) */
  int e = ex - 1;
  if (e < emin) e = emin;
  const double q = ldexp(1.0, e - mant);
  const double r = nearbyint((double)x / q) * q;
  if (fabs(r) > maxfin) return x > 0 ? INFINITY : -INFINITY;
  return (float)r;
}

#define ORACLE_FMT_BF16 1
#define ORACLE_FMT_F16 2

static float round_fmt(float x, int fmt) {
  if (fmt == ORACLE_FMT_BF16) return round_narrow(x, 7, -126, ldexp(2.0 - ldexp(1.0, -7), 127));
  return round_narrow(x, 10, -14, 65504.0);
}

/* out[i] = in[i] rounded to format `fmt` (1: bfloat16, 2: binary16), as a
 * float holding the exact value. */
int oracle_round_to_format(int64_t n, const float *in, float *out, int fmt) {
  if (n < 0 || (n > 0 && (!in || !out)) || (fmt != ORACLE_FMT_BF16 && fmt != ORACLE_FMT_F16))
    return ORACLE_EINVAL;
  for (int64_t i = 0; i < n; ++i) out[i] = round_fmt(in[i], fmt);
  return ORACLE_OK;
}

/* One float step of the canonical expression on zero-padded arrays
 * (ghost layer included, as in oracle_wave2d_f32 / oracle_wave3d_f32):
 * next = step(prev, cur) over the interior; nz = 0 selects 2D. */
static void step_padded_f32(int64_t nz, int64_t ny, int64_t nx, float r2, const float *prev,
                            const float *cur, float *next, int threads) {
  if (nz == 0) {
    _Pragma("omp parallel for num_threads(threads) schedule(static)")
    for (int64_t i = 0; i < ny; ++i)
      for (int64_t j = 0; j < nx; ++j) {
        const float c = cur[P2(i, j)];
        const float north = cur[P2(i - 1, j)], south = cur[P2(i + 1, j)];
        const float west = cur[P2(i, j - 1)], east = cur[P2(i, j + 1)];
        const float sum = (north + south) + (west + east);
        const float lap = sum - 4.0f * c;
        next[P2(i, j)] = fmaf(r2, lap, 2.0f * c - prev[P2(i, j)]);
      }
    return;
  }
  _Pragma("omp parallel for num_threads(threads) schedule(static)")
  for (int64_t z = 0; z < nz; ++z)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        const float c = cur[P3(z, y, x)];
        const float below = cur[P3(z - 1, y, x)], above = cur[P3(z + 1, y, x)];
        const float north = cur[P3(z, y - 1, x)], south = cur[P3(z, y + 1, x)];
        const float west = cur[P3(z, y, x - 1)], east = cur[P3(z, y, x + 1)];
        const float sum = ((below + above) + (north + south)) + (west + east);
        const float lap = sum - 6.0f * c;
        next[P3(z, y, x)] = fmaf(r2, lap, 2.0f * c - prev[P3(z, y, x)]);
      }
}

/* Leapfrog with the fields stored in a 16-bit format and float arithmetic,
 * `depth` steps per pass over the stored fields: the inputs are rounded to
 * the format; each pass takes the stored (u^{n-1}, u^n), applies
 * tb = min(depth, steps left) float steps of the canonical expression
 * (unrounded in between), and stores u^{n+tb-1} and u^{n+tb} rounded to
 * the format.  nz = 0 selects 2D (ny x nx), else 3D (nz x ny x nx). */
int oracle_wave_stored(int64_t nz, int64_t ny, int64_t nx, float r2, int64_t steps,
                       int64_t depth, int fmt, const float *u_prev0, const float *u_cur0,
                       float *u_prev_out, float *u_cur_out, int threads) {
  if (nz < 0 || ny < 1 || nx < 1 || steps < 0 || depth < 1 || !u_prev0 || !u_cur0 ||
      !u_prev_out || !u_cur_out || (fmt != ORACLE_FMT_BF16 && fmt != ORACLE_FMT_F16))
    return ORACLE_EINVAL;
  if (threads < 1) threads = 1;
  const int64_t zz = nz > 0 ? nz : 1;
  const size_t npad = (size_t)(nz > 0 ? nz + 2 : 1) * (size_t)(ny + 2) * (size_t)(nx + 2);
  float *prev = (float *)calloc(npad, sizeof(float));
  float *cur = (float *)calloc(npad, sizeof(float));
  float *next = (float *)calloc(npad, sizeof(float));
  if (!prev || !cur || !next) {
    free(prev); free(cur); free(next);
    return ORACLE_ENOMEM;
  }
  /* interior cell q of the unpadded array <-> padded index */
#define PADDED(z, y, x) (nz > 0 ? P3(z, y, x) : P2(y, x))
  for (int64_t z = 0; z < zz; ++z)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        const size_t q = ((size_t)z * (size_t)ny + (size_t)y) * (size_t)nx + (size_t)x;
        prev[PADDED(z, y, x)] = round_fmt(u_prev0[q], fmt);
        cur[PADDED(z, y, x)] = round_fmt(u_cur0[q], fmt);
      }
  for (int64_t done = 0; done < steps;) {
    const int64_t tb = steps - done < depth ? steps - done : depth;
    for (int64_t s = 0; s < tb; ++s) {
      step_padded_f32(nz, ny, nx, r2, prev, cur, next, threads);
      float *t = prev; prev = cur; cur = next; next = t;
    }
    _Pragma("omp parallel for num_threads(threads) schedule(static)")
    for (int64_t zy = 0; zy < zz * ny; ++zy) {
      const int64_t z = zy / ny, y = zy % ny;
      for (int64_t x = 0; x < nx; ++x) {
        prev[PADDED(z, y, x)] = round_fmt(prev[PADDED(z, y, x)], fmt);
        cur[PADDED(z, y, x)] = round_fmt(cur[PADDED(z, y, x)], fmt);
      }
    }
    done += tb;
  }
  for (int64_t z = 0; z < zz; ++z)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        const size_t q = ((size_t)z * (size_t)ny + (size_t)y) * (size_t)nx + (size_t)x;
        u_prev_out[q] = prev[PADDED(z, y, x)];
        u_cur_out[q] = cur[PADDED(z, y, x)];
      }
#undef PADDED
  free(prev); free(cur); free(next);
  return ORACLE_OK;
}

/* -------------------------------------------------------------- energy -- */

/* Kahan-compensated accumulator. */
typedef struct { double s, c; } ksum;
static void kadd(ksum *k, double v) {
  double y = v - k->c;
  double t = k->s + y;
  k->c = (t - k->s) - y;
  k->s = t;
}

static double get3(const double *u, int64_t nz, int64_t ny, int64_t nx,
                   int64_t z, int64_t y, int64_t x) {
  if (z < 0 || z >= nz || y < 0 || y >= ny || x < 0 || x >= nx) return 0.0;
  return u[((size_t)z * (size_t)ny + (size_t)y) * (size_t)nx + (size_t)x];
}

/* E^{n+1/2} for a 1D, 2D or 3D grid given as nz x ny x nx (use 1 for the
 * missing leading axes).  `u_new` = u^{n+1}, `u_old` = u^n.  The edge sum runs
 * over every pair of face-adjacent cells of the padded box [-1, n_d] along
 * each axis whose extent is not the unit placeholder (the ghost-ghost pairs
 * contribute zero).  `active` says which axes carry the stencil. */
static double energy_any(const double *u_new, const double *u_old, int64_t nz,
                         int64_t ny, int64_t nx, double r2, const int active[3]) {
  ksum kin = {0, 0}, pot = {0, 0};
  for (int64_t z = 0; z < nz; ++z)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        double d = get3(u_new, nz, ny, nx, z, y, x) - get3(u_old, nz, ny, nx, z, y, x);
        kadd(&kin, d * d);
      }
  const int64_t lo[3] = {active[0] ? -1 : 0, active[1] ? -1 : 0, active[2] ? -1 : 0};
  const int64_t hi[3] = {active[0] ? nz : nz - 1, active[1] ? ny : ny - 1,
                         active[2] ? nx : nx - 1};
  for (int axis = 0; axis < 3; ++axis) {
    if (!active[axis]) continue;
    for (int64_t z = lo[0]; z <= hi[0]; ++z)
      for (int64_t y = lo[1]; y <= hi[1]; ++y)
        for (int64_t x = lo[2]; x <= hi[2]; ++x) {
          int64_t z2 = z + (axis == 0), y2 = y + (axis == 1), x2 = x + (axis == 2);
          double an = get3(u_new, nz, ny, nx, z, y, x);
          double bn = get3(u_new, nz, ny, nx, z2, y2, x2);
          double ao = get3(u_old, nz, ny, nx, z, y, x);
          double bo = get3(u_old, nz, ny, nx, z2, y2, x2);
          kadd(&pot, (an - bn) * (ao - bo));
        }
  }
  return kin.s + r2 * pot.s;
}

double oracle_energy1d(const double *u_new, const double *u_old, int64_t n, double r2) {
  const int act[3] = {0, 0, 1};
  return energy_any(u_new, u_old, 1, 1, n, r2, act);
}

double oracle_energy2d(const double *u_new, const double *u_old, int64_t ny,
                       int64_t nx, double r2) {
  const int act[3] = {0, 1, 1};
  return energy_any(u_new, u_old, 1, ny, nx, r2, act);
}

double oracle_energy3d(const double *u_new, const double *u_old, int64_t nz,
                       int64_t ny, int64_t nx, double r2) {
  const int act[3] = {1, 1, 1};
  return energy_any(u_new, u_old, nz, ny, nx, r2, act);
}

/* --------------------------------------------------------------- SAXPY -- */

int oracle_saxpy_f32(int64_t n, float a, const float *x, const float *y, float *z) {
  if (n < 0 || (n > 0 && (!x || !y || !z))) return ORACLE_EINVAL;
  for (int64_t i = 0; i < n; ++i) z[i] = fmaf(a, x[i], y[i]);
  return ORACLE_OK;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
