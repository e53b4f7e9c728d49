// The per-cell update of the 3D seven-point leapfrog scheme, shared by the
// one-step and the temporally blocked 3D kernels so that both produce
// bitwise equal values.  The paper has no stencil of its own: the scheme is
// the chunk kernel this library stands in for the paper's data-parallel
// kernels (the second-order central-difference leapfrog for u_tt = c^2
// lap u, with r2 = (c dt / dx)^2).
#pragma once

#include <hip/hip_runtime.h>

namespace ccl {

// s = ((Z- + Z+) + (Y- + Y+)) + (X- + X+); lap = s - 6C; u+ = fma(r2, lap, 2C - P).
// 6C is rounded (6 needs two significant bits), so it stays a separate
// multiply; 2C is exact, so fma(2, C, -P) equals the rounded 2C - P.
// F is float or double (the arithmetic type).
__device__ __forceinline__ float fma3(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma3(double a, double b, double c) { return fma(a, b, c); }

template <class F>
__device__ __forceinline__ F cell3(F zm, F zp, F ym, F yp, F xm, F xp, F c, F p, F r2) {
  const F sum = ((zm + zp) + (ym + yp)) + (xm + xp);
  const F lap = sum - F(6) * c;
  return fma3(r2, lap, fma3(F(2), c, -p));
}

}  // namespace ccl
