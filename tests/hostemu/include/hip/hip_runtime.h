// Host build of device code, for tests only: a stand-in for the HIP runtime
// header under which a kernel source compiles as plain host C++ (clang,
// -x c++). A launch runs each workgroup's work-items as cooperative fibers
// on the calling thread, one workgroup after another (emu_runtime.cpp):
//   * __syncthreads() waits for every live work-item of the workgroup;
//   * wavefront operations (readlane, shuffles, DPP quad permutes, the
//     16 x 16 matrix-core products) wait for every live lane of the 64-wide
//     wavefront, then compute all lanes' results at once from the lanes'
//     operands, with the lane layouts the device instructions define;
//   * __shared__ variables are static thread_local (one per host thread,
//     so one per running workgroup).
// Lanes of one wavefront do not run in lockstep between wavefront
// operations, so code that passes data between lanes through memory
// without a barrier would be caught as a difference, not hidden.
// This header is never used by the library build (hipcc uses the real one).
#pragma once

#include <math.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline __attribute__((always_inline))
#define __noinline__ __attribute__((noinline))
#define __launch_bounds__(...)
#define __shared__ static thread_local

struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned x_ = 1, unsigned y_ = 1, unsigned z_ = 1) : x(x_), y(y_), z(z_) {}
};

enum hipError_t { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorLaunchFailure = 719 };
typedef struct emu_stream *hipStream_t;
typedef struct emu_event *hipEvent_t;

namespace emu {

struct Index {
  unsigned x, y, z;
};

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

void sync_threads(const char *file, int line);
// Every live lane of the calling wavefront passes `nin` bytes; once all have
// arrived, fn(ins, outs, ctx) runs once and each lane receives its `nout`
// bytes of outs. Slots are 64 bytes.
typedef void (*WaveFn)(const unsigned char (*ins)[64], unsigned char (*outs)[64], int ctx);
void wave_op(WaveFn fn, int ctx, const void *in, size_t nin, void *out, size_t nout);

void op_readlane(const unsigned char (*ins)[64], unsigned char (*outs)[64], int src);
void op_shfl_xor(const unsigned char (*ins)[64], unsigned char (*outs)[64], int mask);
void op_quad_perm(const unsigned char (*ins)[64], unsigned char (*outs)[64], int ctrl);
void op_mfma_f64_16x16x4(const unsigned char (*ins)[64], unsigned char (*outs)[64], int);
void op_mfma_f32_16x16x4(const unsigned char (*ins)[64], unsigned char (*outs)[64], int);
void op_mfma_f32_16x16x32_bf16(const unsigned char (*ins)[64], unsigned char (*outs)[64], int);

template <typename T>
inline T wave_simple(WaveFn fn, int ctx, T v) {
  static_assert(sizeof(T) <= 64, "slot");
  T r;
  wave_op(fn, ctx, &v, sizeof(T), &r, sizeof(T));
  return r;
}

inline int readlane(int v, int src) { return wave_simple(op_readlane, src, v); }
inline int update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl);

// Per-lane operands of the matrix-core products (one 64-byte slot each).
struct InF64 {
  double a, b;
  d4 c;
};
struct InF32 {
  float a, b;
  f4 c;
};
struct InBF16 {
  bf8 a, b;
  f4 c;
};
static_assert(sizeof(InF64) <= 64 && sizeof(InF32) <= 64 && sizeof(InBF16) <= 64, "slot");

inline d4 mfma_f64_16x16x4(double a, double b, d4 c) {
  InF64 in{a, b, c};
  d4 r;
  wave_op(op_mfma_f64_16x16x4, 0, &in, sizeof(in), &r, sizeof(r));
  return r;
}
inline f4 mfma_f32_16x16x4(float a, float b, f4 c) {
  InF32 in{a, b, c};
  f4 r;
  wave_op(op_mfma_f32_16x16x4, 0, &in, sizeof(in), &r, sizeof(r));
  return r;
}
inline f4 mfma_f32_16x16x32_bf16(bf8 a, bf8 b, f4 c) {
  InBF16 in{a, b, c};
  f4 r;
  wave_op(op_mfma_f32_16x16x32_bf16, 0, &in, sizeof(in), &r, sizeof(r));
  return r;
}

// Only the quad_perm controls (0x00-0xFF) with all rows and banks enabled.
void check_dpp(int ctrl, int row_mask, int bank_mask);
inline int update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
  (void)old;
  (void)bound_ctrl;
  check_dpp(ctrl, row_mask, bank_mask);
  return wave_simple(op_quad_perm, ctrl, src);
}

}  // namespace emu

extern thread_local emu::Index threadIdx, blockIdx, blockDim, gridDim;

#define __syncthreads() ::emu::sync_threads(__FILE__, __LINE__)
#define __builtin_amdgcn_readlane(v, src) ::emu::readlane((v), (src))
// every lane is active where the kernels read the first lane
#define __builtin_amdgcn_readfirstlane(v) ::emu::readlane((v), 0)
#define __builtin_amdgcn_sched_barrier(mask) ((void)0)
#define __builtin_amdgcn_update_dpp(old, src, ctrl, rm, bm, bc) \
  ::emu::update_dpp((old), (src), (ctrl), (rm), (bm), (bc))
#define __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, cbsz, abid, blgp) \
  ::emu::mfma_f64_16x16x4((a), (b), (c))
#define __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, cbsz, abid, blgp) \
  ::emu::mfma_f32_16x16x4((a), (b), (c))
#define __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, cbsz, abid, blgp) \
  ::emu::mfma_f32_16x16x32_bf16((a), (b), (c))

template <typename T>
inline T __shfl_xor(T v, int mask, int width = 64) {
  (void)width;
  return ::emu::wave_simple(::emu::op_shfl_xor, mask, v);
}

inline int __double2loint(double v) {
  uint64_t u;
  std::memcpy(&u, &v, 8);
  return int(uint32_t(u));
}
inline int __double2hiint(double v) {
  uint64_t u;
  std::memcpy(&u, &v, 8);
  return int(uint32_t(u >> 32));
}
inline double __hiloint2double(int hi, int lo) {
  const uint64_t u = (uint64_t(uint32_t(hi)) << 32) | uint32_t(lo);
  double v;
  std::memcpy(&v, &u, 8);
  return v;
}
inline float __int_as_float(int v) {
  float f;
  std::memcpy(&f, &v, 4);
  return f;
}
inline int __float_as_int(float f) {
  int v;
  std::memcpy(&v, &f, 4);
  return v;
}

template <typename T>
inline T atomicAdd(T *p, T v) {
  return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}

#define __HIP_MEMORY_SCOPE_AGENT 0
#define __hip_atomic_load(p, order, scope) __atomic_load_n((p), (order))

// Kernels run to completion inside the launch.
#define hipLaunchKernelGGL(kernel, grid, block, shmem, stream, ...) \
  ::emu::launch(dim3(grid), dim3(block), [&]() { kernel(__VA_ARGS__); })
hipError_t hipGetLastError();

#include <functional>
namespace emu {
void launch(dim3 grid, dim3 block, const std::function<void()> &body);
}
