// 16 x 16 x 4 matrix-core products and wavefront broadcasts in FP64 or FP32,
// for kernels whose arithmetic type is a template parameter (the
// elimination's diagonal blocks, panel solves and sweeps run in FP64 for
// FP64 factors and in FP32 for the FP32 factors of the mixed-precision
// solve).
//
// v_mfma_f64_16x16x4f64 and v_mfma_f32_16x16x4f32 take their operands in
// the same lane order: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16].
// They differ in where the output lands: element v of lane l is column l % 16
// and row l / 16 + 4 v (FP64) or 4 (l / 16) + v (FP32).
#pragma once

#include <hip/hip_runtime.h>

namespace rbt {

template <typename C>
struct Mma16;

template <>
struct Mma16<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ constexpr int row(int lk, int v) { return lk + 4 * v; }
};

template <>
struct Mma16<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ constexpr int row(int lk, int v) { return 4 * lk + v; }
};

// Value of v in lane `src` (uniform) of the wavefront.
__device__ __forceinline__ double wave_bcast(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float wave_bcast(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// v of lane K of each quad, to all four lanes of the quad (DPP quad_perm).
template <int K>
__device__ __forceinline__ double quad_bcast_k(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(unsigned(u)), K * 0x55, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(unsigned(u >> 32)), K * 0x55, 0xF, 0xF, false);
  return __builtin_bit_cast(double,
                            (unsigned long long)(unsigned)lo | ((unsigned long long)(unsigned)hi << 32));
}
template <int K>
__device__ __forceinline__ float quad_bcast_k(float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(v), K * 0x55, 0xF, 0xF, false));
}
template <typename C>
__device__ __forceinline__ C quad_bcast(C v, int k) {  // k: compile-time after unrolling
  switch (k) {
    case 0: return quad_bcast_k<0>(v);
    case 1: return quad_bcast_k<1>(v);
    case 2: return quad_bcast_k<2>(v);
    default: return quad_bcast_k<3>(v);
  }
}

__device__ __forceinline__ double fma_c(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_c(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

}  // namespace rbt
