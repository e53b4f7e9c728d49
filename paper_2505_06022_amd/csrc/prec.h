// Storage and arithmetic types of the wave kernels.
//
// A lane handles one aligned group of NV consecutive columns of a row: 16
// bytes of registers per level (four floats or two doubles).  The group is
// loaded from its buffer as one vector access of NV stored elements and
// widened to the arithmetic type; results are narrowed again when stored.
//   P32 : float in memory and in registers (the default path)
//   P64 : double in memory and in registers
//   PB16: bfloat16 in memory, float arithmetic; stored by rounding to
//         nearest, ties to even (8-byte group loads and stores)
//   PH16: IEEE binary16 in memory, float arithmetic; rounded the same way
// With 16-bit storage only the stored levels are rounded: the levels a pass
// keeps in registers stay float, so results depend on the temporal depth
// (but not on tiling or chunking).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ccl.h"

namespace ccl {

template <class F, int NV>
struct Vec {
  F v[NV];
};

// kBody: rows per unrolled loop body of the out-of-place 2D update (see
// wave2d_tile.h); measured per type on the 8192 x 8192 share.
struct P32 {
  using E = float;  // stored element
  using F = float;  // arithmetic
  static constexpr int NV = 4;
  static constexpr int kBody = 12;
  static constexpr int kDtype = CCL_DTYPE_F32;
  typedef float Raw __attribute__((ext_vector_type(4)));
  __device__ static F widen(E e) { return e; }
  __device__ static E narrow(F f) { return f; }
};

struct P64 {
  using E = double;
  using F = double;
  static constexpr int NV = 2;
  static constexpr int kBody = 3;
  static constexpr int kDtype = CCL_DTYPE_F64;
  typedef double Raw __attribute__((ext_vector_type(2)));
  __device__ static F widen(E e) { return e; }
  __device__ static E narrow(F f) { return f; }
};

struct PB16 {
  using E = uint16_t;  // the upper half of a float's bit pattern
  using F = float;
  static constexpr int NV = 4;
  static constexpr int kBody = 3;
  static constexpr int kDtype = CCL_DTYPE_BF16;
  typedef uint16_t Raw __attribute__((ext_vector_type(4)));
  __device__ static F widen(E e) { return __uint_as_float(static_cast<uint32_t>(e) << 16); }
  // round to nearest, ties to even: add half an ulp of the kept part, less
  // one unless the kept part is odd, then truncate (finite inputs; a
  // carry out of the largest finite value gives infinity, as it must)
  __device__ static E narrow(F f) {
    const uint32_t u = __float_as_uint(f);
    return static_cast<E>((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
  }
};

struct PH16 {
  using E = _Float16;
  using F = float;
  static constexpr int NV = 4;
  static constexpr int kBody = 3;
  static constexpr int kDtype = CCL_DTYPE_F16;
  typedef _Float16 Raw __attribute__((ext_vector_type(4)));
  __device__ static F widen(E e) { return static_cast<float>(e); }
  // v_cvt_f16_f32 (round to nearest even) of the float result.  The empty
  // asm pins the float value first: without it the compiler may fold a
  // float fma and this conversion into one mixed-precision fma that rounds
  // the exact result once to binary16, which differs from rounding the
  // float result (double rounding) in a fraction of cases.
  __device__ static E narrow(F f) {
    asm volatile("" : "+v"(f));
    return static_cast<_Float16>(f);
  }
};

// Cross-lane shifts of one arithmetic value (a double moves as two 32-bit
// halves).  from_left: lane l receives lane l-1's value (wave_shr:1, lane 0
// receives 0); from_right: lane l+1's (wave_shl:1, lane 63 receives 0).
// CTRL_L / CTRL_R select the DPP pattern (wave shifts, or row shifts for
// 16-lane rows).
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

}  // namespace ccl
