// Block triangular solves with a factored kb x kb diagonal block (kb <= 128)
// of the elimination, 16 rows (columns) at a time: the update from the
// blocks already solved runs on the FP64 matrix cores, and each 16 x 16
// diagonal block is solved by plain substitution (one lane per right-hand
// side), so the rounding behaviour is that of ordinary forward/back
// substitution. (Multiplying by explicit inverses of the diagonal blocks,
// even 16 x 16 ones, raised the backward error several-fold on N(0,1)
// matrices with large growth.)
//
// The triangle of op(T) is first staged in LDS as its 36 16 x 16 blocks, so
// the serial substitution reads LDS broadcasts instead of waiting on global
// memory.
//
// Left solves, op(T) X = B in place (B: kb x N):
//   LN  T = L (unit lower)     forward  (panel U12 = L11^-1 A12, L y = b)
//   UN  T = U (upper)          backward (U x = y)
//   UT  T = U^T (lower)        forward  (U^T z = g, adjoint solves)
//   LT  T = L^T (unit upper)   backward (L^T w = z)
//   X_I = T_II \ (B_I - sum_{J before I} T_IJ X_J)
// Each wavefront owns 16 columns of B in an LDS strip; a workgroup of four
// covers 64 columns.
//
// Right solve, X U = B in place (B: M x kb) for the panel L21 = A21 U11^-1:
//   X_J = (B_J - sum_{I<J} X_I U_IJ) / U_JJ
// Each wavefront owns 16 rows of B.
//
// MFMA: v_mfma_f64_16x16x4_f64 with the standard operand order; its output
// element (lane l, v) is row l/16 + 4v, column l % 16.
#include "internal.h"

namespace rbt {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int NB = kNB;  // 128
constexpr int IB = 16;
constexpr int NBK = NB / IB;                 // 8 blocks per side
constexpr int NTRI = NBK * (NBK + 1) / 2;    // 36 blocks in a triangle
constexpr int BLK = IB * IB;                 // 256 doubles per block

template <TriMode MODE>
constexpr bool forward_order() {
  return MODE == TriMode::LN || MODE == TriMode::UT;
}

// (I, J) of staged block b: lower triangle enumerated row by row
// (b = I (I + 1) / 2 + J, J <= I); the upper triangle is its transpose.
struct BlockIJ {
  int i[NTRI], j[NTRI];
};
constexpr BlockIJ lower_blocks() {
  BlockIJ t{};
  int b = 0;
  for (int I = 0; I < NBK; ++I)
    for (int J = 0; J <= I; ++J) {
      t.i[b] = I;
      t.j[b] = J;
      ++b;
    }
  return t;
}
__constant__ constexpr BlockIJ kLower = lower_blocks();

// Index of block (I, J) of the staged triangle: lower (I >= J) for the
// forward modes, upper (I <= J) otherwise.
template <bool LOWER>
__device__ __forceinline__ int tri_index(int I, int J) {
  return LOWER ? I * (I + 1) / 2 + J : J * (J + 1) / 2 + I;
}

// op(T)(i, j) read from global memory (i, j < kb).
template <TriMode MODE>
__device__ __forceinline__ double op_t(const double *T, int64_t ldt, int i, int j) {
  if constexpr (MODE == TriMode::LN || MODE == TriMode::UN)
    return T[i + int64_t(j) * ldt];
  else
    return T[j + int64_t(i) * ldt];
}

// Stage the triangle of op(T) blocks into LDS, each block column-major
// (element (r, c) at c * 16 + r); entries at or beyond kb are zero. Loads
// are issued in batches of 12 blocks before any is stored.
template <TriMode MODE>
__device__ void stage_left(const double *T, int64_t ldt, int kb, double *tri) {
  constexpr bool LOWER = forward_order<MODE>();
  const int r = threadIdx.x % IB, c = threadIdx.x / IB;  // 256 threads = one block
#pragma unroll
  for (int b0 = 0; b0 < NTRI; b0 += 12) {
    double v[12];
#pragma unroll
    for (int u = 0; u < 12; ++u) {
      const int b = b0 + u;
      const int I = LOWER ? kLower.i[b] : kLower.j[b];
      const int J = LOWER ? kLower.j[b] : kLower.i[b];
      const int i = IB * I + r, j = IB * J + c;
      v[u] = (i < kb && j < kb) ? op_t<MODE>(T, ldt, i, j) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 12; ++u) tri[(b0 + u) * BLK + c * IB + r] = v[u];
  }
}

// Load / store a wavefront's 128 x 16 strip of B (column c at strip[row * 16 + c]).
__device__ __forceinline__ void strip_load(double *strip, const double *B, int64_t ldb, int kb,
                                           int64_t col0, int64_t N, int lane) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    double v[16];
#pragma unroll
    for (int c = 0; c < IB; ++c) {
      const int row = lane + 64 * h;
      const int64_t col = col0 + c;
      v[c] = (row < kb && col < N) ? B[row + col * ldb] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < IB; ++c) strip[(lane + 64 * h) * IB + c] = v[c];
  }
}

__device__ __forceinline__ void strip_store(const double *strip, double *B, int64_t ldb, int kb,
                                            int64_t col0, int64_t N, int lane) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int c = 0; c < IB; ++c) {
      const int row = lane + 64 * h;
      const int64_t col = col0 + c;
      if (row < kb && col < N) B[row + col * ldb] = strip[row * IB + c];
    }
  }
}

template <TriMode MODE>
__global__ void __launch_bounds__(256) k_trsm_left(int kb, int64_t N, const double *T,
                                                   int64_t ldt, double *B, int64_t ldb) {
  __shared__ double tri[NTRI * BLK];
  __shared__ double strip_all[4][NB * IB];
  constexpr bool LOWER = forward_order<MODE>();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  double *strip = strip_all[wave];
  const int64_t col0 = int64_t(blockIdx.x) * 64 + wave * 16;

  stage_left<MODE>(T, ldt, kb, tri);
  strip_load(strip, B, ldb, kb, col0, N, lane);
  __syncthreads();

  const int nbk = (kb + IB - 1) / IB;
  for (int step = 0; step < nbk; ++step) {
    const int I = LOWER ? step : nbk - 1 - step;
    d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    for (int s2 = 0; s2 < step; ++s2) {
      const int J = LOWER ? s2 : nbk - 1 - s2;
      const double *tb = tri + tri_index<LOWER>(I, J) * BLK;
#pragma unroll
      for (int kk = 0; kk < 4; kk += 2) {
        const int k0 = 4 * kk + lk, k1 = 4 * (kk + 1) + lk;
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(tb[k0 * IB + l16],
                                                    strip[(IB * J + k0) * IB + l16], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(tb[k1 * IB + l16],
                                                    strip[(IB * J + k1) * IB + l16], acc1, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) strip[(IB * I + lk + 4 * v) * IB + l16] -= acc0[v] + acc1[v];
    __syncthreads();
    // substitution inside the diagonal block: lane c < 16 owns column c
    const int bs = kb - IB * I < IB ? kb - IB * I : IB;
    if (lane < IB) {
      const int o = IB * I;
      const double *tb = tri + tri_index<LOWER>(I, I) * BLK;  // element (i, j) at j*16+i
      double x[IB];
#pragma unroll
      for (int i = 0; i < IB; ++i) x[i] = strip[(o + i) * IB + lane];
      if constexpr (LOWER) {
#pragma unroll
        for (int j = 0; j < IB; ++j) {
          if (j < bs) {
            if constexpr (MODE == TriMode::UT) x[j] = x[j] / tb[j * IB + j];
#pragma unroll
            for (int i = j + 1; i < IB; ++i) x[i] -= tb[j * IB + i] * x[j];
          }
        }
      } else {
#pragma unroll
        for (int j = IB - 1; j >= 0; --j) {
          if (j < bs) {
            if constexpr (MODE == TriMode::UN) x[j] = x[j] / tb[j * IB + j];
#pragma unroll
            for (int i = 0; i < j; ++i) x[i] -= tb[j * IB + i] * x[j];
          }
        }
      }
#pragma unroll
      for (int i = 0; i < IB; ++i) strip[(o + i) * IB + lane] = (i < bs) ? x[i] : 0.0;
    }
    __syncthreads();
  }

  strip_store(strip, B, ldb, kb, col0, N, lane);
}

constexpr int RS = NB + 1;  // row stride of the right-solve strip (odd: conflict-free)

__global__ void __launch_bounds__(256) k_trsm_right_upper(int kb, int64_t M, const double *T,
                                                          int64_t ldt, double *B, int64_t ldb) {
  __shared__ double tri[NTRI * BLK];  // upper blocks of U, each row-major (r * 16 + c)
  __shared__ double strip_all[4][IB * RS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  double *strip = strip_all[wave];
  const int64_t row0 = int64_t(blockIdx.x) * 64 + wave * 16;

  {
    const int r = threadIdx.x % IB, c = threadIdx.x / IB;
#pragma unroll
    for (int b0 = 0; b0 < NTRI; b0 += 12) {
      double v[12];
#pragma unroll
      for (int u = 0; u < 12; ++u) {
        const int b = b0 + u;  // upper block (I, J) = transpose of lower entry b
        const int i = IB * kLower.j[b] + r, j = IB * kLower.i[b] + c;
        v[u] = (i < kb && j < kb) ? T[i + int64_t(j) * ldt] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 12; ++u) tri[(b0 + u) * BLK + r * IB + c] = v[u];
    }
  }
  {
    // strip: 16 rows x 128 columns; lane = (row = lane % 16, column group lane / 16)
    const int r = lane % IB, cg = lane / IB;
    const int64_t row = row0 + r;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int c = cg + 4 * (16 * h + u);
        v[u] = (row < M && c < kb) ? B[row + int64_t(c) * ldb] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) strip[r * RS + cg + 4 * (16 * h + u)] = v[u];
    }
  }
  __syncthreads();

  const int nbk = (kb + IB - 1) / IB;
  for (int J = 0; J < nbk; ++J) {
    d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    for (int I = 0; I < J; ++I) {
      const double *tb = tri + tri_index<false>(I, J) * BLK;
#pragma unroll
      for (int kk = 0; kk < 4; kk += 2) {
        const int k0 = 4 * kk + lk, k1 = 4 * (kk + 1) + lk;
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(strip[l16 * RS + IB * I + k0],
                                                    tb[k0 * IB + l16], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(strip[l16 * RS + IB * I + k1],
                                                    tb[k1 * IB + l16], acc1, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) strip[(lk + 4 * v) * RS + IB * J + l16] -= acc0[v] + acc1[v];
    __syncthreads();
    // substitution inside the diagonal block: lane r < 16 owns row r
    const int bs = kb - IB * J < IB ? kb - IB * J : IB;
    if (lane < IB) {
      const int o = IB * J;
      const double *tb = tri + tri_index<false>(J, J) * BLK;  // element (r, c) at r*16+c
      double x[IB];
#pragma unroll
      for (int c = 0; c < IB; ++c) x[c] = strip[lane * RS + o + c];
#pragma unroll
      for (int c = 0; c < IB; ++c) {
        if (c < bs) {
          x[c] = x[c] / tb[c * IB + c];
#pragma unroll
          for (int c2 = c + 1; c2 < IB; ++c2) x[c2] -= x[c] * tb[c * IB + c2];
        }
      }
#pragma unroll
      for (int c = 0; c < IB; ++c) strip[lane * RS + o + c] = (c < bs) ? x[c] : 0.0;
    }
    __syncthreads();
  }

  {
    const int r = lane % IB, cg = lane / IB;
    const int64_t row = row0 + r;
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const int c = cg + 4 * u;
      if (row < M && c < kb) B[row + int64_t(c) * ldb] = strip[r * RS + c];
    }
  }
}

}  // namespace

hipError_t launch_trsm_left(TriMode mode, int kb, int64_t N, const double *T, int64_t ldt,
                            double *B, int64_t ldb, hipStream_t s) {
  if (kb <= 0 || N <= 0) return hipSuccess;
  if (kb > kNB) return hipErrorInvalidValue;
  const dim3 grid(unsigned((N + 63) / 64));
  switch (mode) {
    case TriMode::LN: hipLaunchKernelGGL(k_trsm_left<TriMode::LN>, grid, dim3(256), 0, s, kb, N, T, ldt, B, ldb); break;
    case TriMode::UN: hipLaunchKernelGGL(k_trsm_left<TriMode::UN>, grid, dim3(256), 0, s, kb, N, T, ldt, B, ldb); break;
    case TriMode::UT: hipLaunchKernelGGL(k_trsm_left<TriMode::UT>, grid, dim3(256), 0, s, kb, N, T, ldt, B, ldb); break;
    case TriMode::LT: hipLaunchKernelGGL(k_trsm_left<TriMode::LT>, grid, dim3(256), 0, s, kb, N, T, ldt, B, ldb); break;
  }
  return hipGetLastError();
}

hipError_t launch_trsm_right_upper(int kb, int64_t M, const double *T, int64_t ldt, double *B,
                                   int64_t ldb, hipStream_t s) {
  if (kb <= 0 || M <= 0) return hipSuccess;
  if (kb > kNB) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_trsm_right_upper, dim3(unsigned((M + 63) / 64)), dim3(256), 0, s, kb, M,
                     T, ldt, B, ldb);
  return hipGetLastError();
}

}  // namespace rbt
