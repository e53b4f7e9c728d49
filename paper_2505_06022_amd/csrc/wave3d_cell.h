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
__device__ __forceinline__ float cell3(float zm, float zp, float ym, float yp, float xm, float xp,
                                       float c, float p, float r2) {
  const float sum = ((zm + zp) + (ym + yp)) + (xm + xp);
  const float lap = sum - 6.0f * c;
  return fmaf(r2, lap, fmaf(2.0f, c, -p));
}

}  // namespace ccl
