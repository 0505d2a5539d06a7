// Diagonal-block kernel of the blocked elimination without pivoting.
//
// One workgroup of 1024 threads factors a kb x kb diagonal block
// (kb <= 128) in place, A = L U with unit-lower L (Sec. 1, step 2: GENP),
// then inverts both triangles and writes them, packed, to Winv:
// strictly below the diagonal L^-1 (its unit diagonal implied), on and above
// the diagonal U^-1. The inverses turn the panel and right-hand-side
// triangular solves into matrix-core GEMMs (k_gemm.hip).
//
// Layout: thread t owns row r = t % 128 and the 16 columns l = g + 8 j,
// g = t / 128, j = 0..15, in registers. A wavefront therefore holds 64 rows
// of the same column set, so the pivot-row values it reads from LDS are
// broadcasts and its loads/stores are contiguous column runs.
//
// Step c of the elimination: the owners of row c publish it, the owners of
// column c publish the column; after one barrier every thread scales its
// multiplier and updates its 16 entries (right-looking, rank-1). Buffers are
// double-buffered by step parity, so one barrier per step suffices.
//
// Inversion (after the factorization), both triangles in one loop of kb
// steps, again rank-1 and right-looking:
//   U^-1: X = I; for c = kb-1 .. 0: X[c,:] /= U[c,c]; X[r,:] -= U[r,c] X[c,:], r < c
//   L^-1: Y = I; for c = 0 .. kb-1:                   Y[r,:] -= L[r,c] Y[c,:], r > c
// A zero pivot is recorded in *info (first one, 1-based, offset gofs) and the
// arithmetic continues with IEEE Inf/NaN.
#include "internal.h"

namespace rbt {

namespace {

constexpr int NT = 1024;
constexpr int NB = kNB;  // 128
constexpr int NJ = NB / 8;

__global__ void __launch_bounds__(NT) k_diag_lu(int kb, double *__restrict__ A, int64_t lda,
                                                 double *__restrict__ W, int64_t gofs,
                                                 int32_t *__restrict__ info) {
  __shared__ double rowbuf[2][NB];
  __shared__ double colbuf[2][NB];
  __shared__ double rowbuf2[2][NB];
  __shared__ double colbuf2[2][NB];
  __shared__ double diag[NB];

  const int t = threadIdx.x;
  const int r = t % NB;
  const int g = t / NB;
  const bool rok = r < kb;

  double S[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int l = g + 8 * j;
    S[j] = (rok && l < kb) ? A[r + int64_t(l) * lda] : 0.0;
  }

  // ---- factorization ----
  for (int c = 0; c < kb; ++c) {
    const int b = c & 1;
    const int gc = c & 7, jc = c >> 3;
    if (r == c) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) rowbuf[b][g + 8 * j] = S[j];
    }
    if (g == gc) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        if (j == jc) v = S[j];
      colbuf[b][r] = v;
    }
    __syncthreads();
    const double p = rowbuf[b][c];
    if (t == 0 && p == 0.0 && info != nullptr) atomicCAS(info, 0, int32_t(gofs + c + 1));
    if (r > c) {
      const double lr = colbuf[b][r] / p;
      if (g == gc) {
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          if (j == jc) S[j] = lr;
      }
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int l = g + 8 * j;
        if (l > c) S[j] -= lr * rowbuf[b][l];
      }
    }
  }

  // write the factors back
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int l = g + 8 * j;
    if (rok && l < kb) A[r + int64_t(l) * lda] = S[j];
  }

  // ---- inversion of both triangles ----
  if (g == (r & 7)) {
    double v = 1.0;
#pragma unroll
    for (int j = 0; j < NJ; ++j)
      if (j == (r >> 3)) v = S[j];
    diag[r] = rok ? v : 1.0;
  }
  double X[NJ], Y[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int l = g + 8 * j;
    X[j] = (l == r) ? 1.0 : 0.0;
    Y[j] = X[j];
  }
  __syncthreads();

  for (int s = 0; s < kb; ++s) {
    const int b = s & 1;
    const int cu = kb - 1 - s;  // U^-1 step (descending)
    const int cl = s;           // L^-1 step (ascending)
    if (r == cu) {
      const double dinv = diag[cu];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        X[j] = X[j] / dinv;
        rowbuf[b][g + 8 * j] = X[j];
      }
    }
    if (r == cl) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) rowbuf2[b][g + 8 * j] = Y[j];
    }
    if (g == (cu & 7)) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        if (j == (cu >> 3)) v = S[j];
      colbuf[b][r] = v;  // U[r, cu] (used for r < cu)
    }
    if (g == (cl & 7)) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        if (j == (cl >> 3)) v = S[j];
      colbuf2[b][r] = v;  // L[r, cl] (used for r > cl)
    }
    __syncthreads();
    if (r < cu) {
      const double u = colbuf[b][r];
#pragma unroll
      for (int j = 0; j < NJ; ++j) X[j] -= u * rowbuf[b][g + 8 * j];
    }
    if (r > cl && r < kb) {
      const double lv = colbuf2[b][r];
#pragma unroll
      for (int j = 0; j < NJ; ++j) Y[j] -= lv * rowbuf2[b][g + 8 * j];
    }
  }

  // packed inverse: strict lower from Y, upper (with diagonal) from X
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int l = g + 8 * j;
    if (rok && l < kb) W[r + int64_t(l) * NB] = (r > l) ? Y[j] : X[j];
  }
}

}  // namespace

hipError_t launch_diag_lu(int kb, double *A, int64_t lda, double *Winv, int64_t gofs,
                          int32_t *info, hipStream_t s) {
  if (kb <= 0) return hipSuccess;
  if (kb > kNB) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_diag_lu, dim3(1), dim3(NT), 0, s, kb, A, lda, Winv, gofs, info);
  return hipGetLastError();
}

}  // namespace rbt
