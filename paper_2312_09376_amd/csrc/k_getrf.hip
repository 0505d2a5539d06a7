// Diagonal-block kernel of the blocked elimination without pivoting.
//
// One workgroup of 256 threads factors a kb x kb diagonal block (kb <= 128)
// in place, A = L U with unit-lower L (Sec. 1, step 2: GENP). The block is
// held in LDS (column-major, leading dimension 129 so that row-wise and
// column-wise lane patterns are both bank-conflict free) and eliminated in
// eight 16-column steps:
//   1. the 16-column panel is factored right-looking, rank-1, by wavefront 0
//      alone: lane l holds rows l and l + 64 of the panel in registers and
//      each pivot row is broadcast with readlane, so the 16 steps need no
//      workgroup barrier;
//   2. the 16-row block of U to its right is solved by forward substitution
//      with the panel's unit-lower 16 x 16 block (one lane per column);
//   3. the trailing block takes a rank-16 update on the FP64 matrix cores,
//      16 x 16 tiles shared out over the four wavefronts; each tile's
//      accumulator starts from the LDS values and the L operand is negated.
// Rows and columns beyond kb hold the identity, so they never disturb the
// active part. The block may be stored in FP32 (mixed-precision elimination):
// it is then widened on load, eliminated in FP64 and rounded once on store. A zero pivot is recorded in *info (first one, 1-based, offset
// gofs) and the arithmetic continues with IEEE Inf/NaN.
#include "internal.h"

namespace rbt {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int NB = kNB;  // 128
constexpr int LD = NB + 1;
constexpr int PW = 16;   // panel width

// Value of v in lane `src` (uniform) of the wavefront.
__device__ __forceinline__ double wave_bcast(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

template <typename T>
__global__ void __launch_bounds__(256) k_diag_lu(int kb, T *__restrict__ A, int64_t lda,
                                                 int64_t gofs, int32_t *__restrict__ info) {
  __shared__ double S[NB * LD];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lk = lane >> 4;

  // Staging: every load of a batch is issued before any is consumed, so the
  // batch costs one memory latency instead of one per element.
  {
    const int r = tid & (NB - 1), c0 = tid >> 7;  // row, first column (0/1)
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      // unconditional loads at clamped valid indices, masked afterwards
      T v[32];
      const int rr = r < kb ? r : kb - 1;
#pragma unroll
      for (int i = 0; i < 32; ++i) {
        const int c = c0 + 2 * (32 * half + i);
        v[i] = A[rr + int64_t(c < kb ? c : kb - 1) * lda];
      }
#pragma unroll
      for (int i = 0; i < 32; ++i) {
        const int c = c0 + 2 * (32 * half + i);
        S[c * LD + r] = (r < kb && c < kb) ? double(v[i]) : ((r == c) ? 1.0 : 0.0);
      }
    }
  }
  __syncthreads();

  for (int c0 = 0; c0 < kb; c0 += PW) {
    // ---- 1. panel factorization (rows >= c0, columns c0..c0+15), wave 0 ----
    if (wave == 0) {
      double xa[PW], xb[PW];  // rows lane and lane + 64
#pragma unroll
      for (int j = 0; j < PW; ++j) {
        xa[j] = S[(c0 + j) * LD + lane];
        xb[j] = S[(c0 + j) * LD + lane + 64];
      }
#pragma unroll
      for (int cc = 0; cc < PW; ++cc) {
        const int c = c0 + cc;
        const int owner = c & 63;
        const bool upper = c >= 64;
        double prow[PW];
#pragma unroll
        for (int j = cc; j < PW; ++j) prow[j] = wave_bcast(upper ? xb[j] : xa[j], owner);
        const double p = prow[cc];
        if (lane == 0 && c < kb && p == 0.0 && info != nullptr)
          atomicCAS(info, 0, int32_t(gofs + c + 1));
        const bool acta = lane > c, actb = lane + 64 > c;
        const double rp = 1.0 / p;  // one division per pivot (scaling as in LAPACK's getf2)
        const double la = xa[cc] * rp, lb = xb[cc] * rp;
        xa[cc] = acta ? la : xa[cc];
        xb[cc] = actb ? lb : xb[cc];
#pragma unroll
        for (int j = cc + 1; j < PW; ++j) {
          const double ua = xa[j] - la * prow[j];
          const double ub = xb[j] - lb * prow[j];
          xa[j] = acta ? ua : xa[j];
          xb[j] = actb ? ub : xb[j];
        }
      }
#pragma unroll
      for (int j = 0; j < PW; ++j) {
        if (lane >= c0) S[(c0 + j) * LD + lane] = xa[j];
        if (lane + 64 >= c0) S[(c0 + j) * LD + lane + 64] = xb[j];
      }
    }
    __syncthreads();

    const int c1 = c0 + PW;  // first column/row after the panel
    if (c1 >= NB) break;
    // ---- 2. U block row: rows c0..c0+15, columns c1..127 ----
    if (tid < NB - c1) {
      const int col = c1 + tid;
      double y[PW];
#pragma unroll
      for (int i = 0; i < PW; ++i) y[i] = S[col * LD + c0 + i];
#pragma unroll
      for (int i = 0; i < PW; ++i)
#pragma unroll
        for (int i2 = i + 1; i2 < PW; ++i2) y[i2] -= S[(c0 + i) * LD + c0 + i2] * y[i];
#pragma unroll
      for (int i = 0; i < PW; ++i) S[col * LD + c0 + i] = y[i];
    }
    __syncthreads();
    // ---- 3. trailing rank-16 update on 16 x 16 tiles ----
    const int nt = (NB - c1) / PW;
    for (int t = wave; t < nt * nt; t += 4) {
      const int i0 = c1 + PW * (t % nt), j0 = c1 + PW * (t / nt);
      d4 acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = S[(j0 + l16) * LD + i0 + lk + 4 * v];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int k = c0 + 4 * kk + lk;
        const double a = -S[k * LD + i0 + l16];
        const double bv = S[(j0 + l16) * LD + k];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) S[(j0 + l16) * LD + i0 + lk + 4 * v] = acc[v];
    }
    __syncthreads();
  }

  {
    const int rr = tid & (NB - 1), c0 = tid >> 7;
#pragma unroll 16
    for (int i = 0; i < 64; ++i) {
      const int c = c0 + 2 * i;
      if (rr < kb && c < kb) A[rr + int64_t(c) * lda] = T(S[c * LD + rr]);
    }
  }
}

}  // namespace

template <typename T>
hipError_t diag_lu_t(int kb, T *A, int64_t lda, int64_t gofs, int32_t *info, hipStream_t s) {
  if (kb <= 0) return hipSuccess;
  if (kb > kNB) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_diag_lu<T>, dim3(1), dim3(256), 0, s, kb, A, lda, gofs, info);
  return hipGetLastError();
}

hipError_t launch_diag_lu(int kb, double *A, int64_t lda, int64_t gofs, int32_t *info,
                          hipStream_t s) {
  return diag_lu_t(kb, A, lda, gofs, info, s);
}
hipError_t launch_diag_lu(int kb, float *A, int64_t lda, int64_t gofs, int32_t *info,
                          hipStream_t s) {
  return diag_lu_t(kb, A, lda, gofs, info, s);
}

}  // namespace rbt
