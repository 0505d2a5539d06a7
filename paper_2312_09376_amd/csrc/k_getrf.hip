// Diagonal-block kernel of the blocked elimination without pivoting.
//
// One workgroup of 1024 threads factors a kb x kb diagonal block
// (kb <= 128) in place, A = L U with unit-lower L (Sec. 1, step 2: GENP).
// The off-diagonal panels are then solved against it by k_trsm.hip.
//
// Layout: thread t owns row r = t % 128 and the 16 columns l = g + 8 j,
// g = t / 128, j = 0..15, in registers. A wavefront holds 64 rows of one
// column set, so pivot-row reads from LDS are broadcasts and its global
// loads/stores are contiguous column runs.
//
// Step c of the elimination: the owners of row c publish it, the owners of
// column c publish the column; after one barrier every thread below row c
// scales its multiplier and updates its 16 entries (right-looking, rank-1),
// the update of already-final columns being discarded by a select (no
// branches). Buffers alternate by step parity, so one barrier per step.
//
// A zero pivot is recorded in *info (first one, 1-based, offset gofs) and the
// arithmetic continues with IEEE Inf/NaN.
#include "internal.h"

namespace rbt {

namespace {

constexpr int NT = 1024;
constexpr int NB = kNB;  // 128
constexpr int NJ = NB / 8;

__global__ void __launch_bounds__(NT) k_diag_lu(int kb, double *__restrict__ A, int64_t lda,
                                                 int64_t gofs, int32_t *__restrict__ info) {
  __shared__ double rowbuf[2][NB];
  __shared__ double colbuf[2][NB];

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
      for (int j = 0; j < NJ; ++j) v = (j == jc) ? S[j] : v;
      colbuf[b][r] = v;
    }
    __syncthreads();
    const double p = rowbuf[b][c];
    if (t == 0 && p == 0.0 && info != nullptr) atomicCAS(info, 0, int32_t(gofs + c + 1));
    if (r > c) {
      const double lr = colbuf[b][r] / p;
      double rv[NJ];
#pragma unroll
      for (int j = 0; j < NJ; ++j) rv[j] = rowbuf[b][g + 8 * j];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int l = g + 8 * j;
        const double upd = S[j] - lr * rv[j];
        S[j] = (l > c) ? upd : ((l == c) ? lr : S[j]);
      }
    }
  }

#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int l = g + 8 * j;
    if (rok && l < kb) A[r + int64_t(l) * lda] = S[j];
  }

}

}  // namespace

hipError_t launch_diag_lu(int kb, double *A, int64_t lda, int64_t gofs, int32_t *info,
                          hipStream_t s) {
  if (kb <= 0) return hipSuccess;
  if (kb > kNB) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_diag_lu, dim3(1), dim3(NT), 0, s, kb, A, lda, gofs, info);
  return hipGetLastError();
}

}  // namespace rbt
