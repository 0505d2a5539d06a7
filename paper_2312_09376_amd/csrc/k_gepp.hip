// Gaussian elimination with partial pivoting (GEPP), the robust solver that
// the fallback of Sec. 5 re-solves with when the unpivoted RBT solve cannot
// be refined to the tolerance (the "responsibly reckless" pairing of a fast
// unpivoted solve with a check and a pivoted re-solve).
//
// Blocked right-looking, panels of kNB = 128 columns:
//   for each column j of the panel:
//     k_pivot_partial  many workgroups: max |a_ij| over their rows i >= j
//                      (first index among equal magnitudes, as LAPACK's
//                      idamax);
//     k_pivot_swap     one workgroup: reduces the partial maxima to the pivot
//                      row p, records ipiv[j] = p + 1 (1-based, LAPACK's
//                      getrf convention) and swaps rows j and p over all n
//                      columns (so the L part, the panel and the trailing
//                      matrix are permuted at once);
//     k_panel_column   many workgroups, one row per thread: l_ij = a_ij / a_jj
//                      and the rank-1 update of the panel's columns right of
//                      j (rows below j); coalesced along the rows;
//   then U12 = L11^-1 A12 (k_trsm.hip, unit lower) and A22 -= L21 U12 on the
//   FP64 matrix cores (k_gemm.hip).
// A zero pivot column (max |a_ij| = 0) is recorded in *info (first, 1-based)
// and left unswapped; the elimination goes on with IEEE Inf/NaN.
//
// Solves: ipiv is turned into the permutation it applies (one thread,
// sequential, in LDS), the rows of B are gathered through it in parallel, and
// the triangular solves reuse the sweeps of the unpivoted factors (the L\U
// layout is the same).
#include "internal.h"

namespace rbt {

namespace {

constexpr int TPB = 256;
constexpr int kPivotGroups = 256;  // workgroups of the pivot search

__device__ __forceinline__ bool better(double v, int64_t i, double bv, int64_t bi) {
  // larger magnitude wins; equal magnitudes: the smaller row index; NaN
  // never wins over a number (a NaN column then pivots on its first row)
  return v > bv || (v == bv && i < bi);
}

__global__ void __launch_bounds__(TPB)
    k_pivot_partial(int64_t n, const double *__restrict__ A, int64_t lda, int64_t j,
                    double *__restrict__ pval, int64_t *__restrict__ pidx) {
  __shared__ double sv[TPB / 64];
  __shared__ int64_t si[TPB / 64];
  double bv = -1.0;
  int64_t bi = INT64_MAX;
  const double *col = A + j * lda;
  for (int64_t i = j + int64_t(blockIdx.x) * TPB + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * TPB) {
    const double v = fabs(col[i]);
    if (better(v, i, bv, bi)) {
      bv = v;
      bi = i;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(bv, o);
    const int64_t oi = __shfl_xor(bi, o);
    if (better(ov, oi, bv, bi)) {
      bv = ov;
      bi = oi;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sv[wave] = bv;
    si[wave] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < TPB / 64; ++w)
      if (better(sv[w], si[w], bv, bi)) {
        bv = sv[w];
        bi = si[w];
      }
    pval[blockIdx.x] = bv;
    pidx[blockIdx.x] = bi;
  }
}

__global__ void __launch_bounds__(TPB)
    k_pivot_swap(int64_t n, double *__restrict__ A, int64_t lda, int64_t j, int groups,
                 const double *__restrict__ pval, const int64_t *__restrict__ pidx,
                 int64_t *__restrict__ ipiv, int32_t *__restrict__ info) {
  __shared__ int64_t p_sh;
  if (threadIdx.x == 0) {
    double bv = -1.0;
    int64_t bi = INT64_MAX;
    for (int g = 0; g < groups; ++g)
      if (better(pval[g], pidx[g], bv, bi)) {
        bv = pval[g];
        bi = pidx[g];
      }
    int64_t p = bi;
    if (!(bv > 0.0) || p >= n) {  // zero (or NaN) column: no interchange
      if (bv == 0.0 && info != nullptr && *info == 0) *info = int32_t(j + 1);
      p = j;
    }
    ipiv[j] = p + 1;
    p_sh = p;
  }
  __syncthreads();
  const int64_t p = p_sh;
  if (p == j) return;
  for (int64_t c = threadIdx.x; c < n; c += TPB) {
    double *a = A + j + c * lda, *b = A + p + c * lda;
    const double t = *a;
    *a = *b;
    *b = t;
  }
}

// Column j of the panel [k0, kend): multipliers below the pivot and the
// rank-1 update of the panel columns j+1 .. kend-1.
__global__ void __launch_bounds__(TPB)
    k_panel_column(int64_t n, double *__restrict__ A, int64_t lda, int64_t j, int64_t kend) {
  const int64_t i = j + 1 + int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (i >= n) return;
  const double piv = A[j + j * lda];
  const double l = A[i + j * lda] / piv;
  A[i + j * lda] = l;
  for (int64_t c = j + 1; c < kend; ++c) A[i + c * lda] -= l * A[j + c * lda];
}

// perm[i] = original row that ends in row i after the interchanges
// ipiv[0..n) (1-based), applied in order.
__global__ void __launch_bounds__(64)
    k_ipiv_to_perm(int64_t n, const int64_t *__restrict__ ipiv, int64_t *__restrict__ perm) {
  extern __shared__ int32_t p_lds[];
  const bool in_lds = n <= kPermLdsMax;
  for (int64_t i = threadIdx.x; i < n; i += 64) {
    if (in_lds)
      p_lds[i] = int32_t(i);
    else
      perm[i] = i;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int64_t j = 0; j < n; ++j) {
      const int64_t p = ipiv[j] - 1;
      if (p == j || p < 0 || p >= n) continue;
      if (in_lds) {
        const int32_t t = p_lds[j];
        p_lds[j] = p_lds[p];
        p_lds[p] = t;
      } else {
        const int64_t t = perm[j];
        perm[j] = perm[p];
        perm[p] = t;
      }
    }
  }
  __syncthreads();
  if (in_lds)
    for (int64_t i = threadIdx.x; i < n; i += 64) perm[i] = p_lds[i];
}

// Y[i, c] = B[perm[i], c]
__global__ void __launch_bounds__(TPB)
    k_gather_rows(int64_t n, int64_t nrhs, const int64_t *__restrict__ perm,
                  const double *__restrict__ B, int64_t ldb, double *__restrict__ Y,
                  int64_t ldy) {
  const int64_t i = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (i >= n) return;
  const int64_t r = perm[i];
  for (int64_t c = blockIdx.y; c < nrhs; c += gridDim.y) Y[i + c * ldy] = B[r + c * ldb];
}

}  // namespace

size_t gepp_scratch_bytes() {
  return align256(size_t(kPivotGroups) * sizeof(double)) +
         align256(size_t(kPivotGroups) * sizeof(int64_t));
}

hipError_t launch_gepp(int64_t n, double *A, int64_t lda, int64_t *ipiv, int32_t *info,
                       void *scratch, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  double *pval = static_cast<double *>(scratch);
  int64_t *pidx = reinterpret_cast<int64_t *>(static_cast<char *>(scratch) +
                                              align256(size_t(kPivotGroups) * sizeof(double)));
  for (int64_t k0 = 0; k0 < n; k0 += kNB) {
    const int64_t kend = k0 + kNB < n ? k0 + kNB : n;
    const int kb = int(kend - k0);
    for (int64_t j = k0; j < kend; ++j) {
      const int64_t rows = n - j;
      const int groups = int(rows > int64_t(kPivotGroups) * TPB
                                 ? kPivotGroups
                                 : (rows + TPB - 1) / TPB);
      hipLaunchKernelGGL(k_pivot_partial, dim3(unsigned(groups)), dim3(TPB), 0, s, n, A, lda, j,
                         pval, pidx);
      hipLaunchKernelGGL(k_pivot_swap, dim3(1), dim3(TPB), 0, s, n, A, lda, j, groups, pval,
                         pidx, ipiv, info);
      if (rows > 1)
        hipLaunchKernelGGL(k_panel_column, dim3(unsigned((rows - 1 + TPB - 1) / TPB)), dim3(TPB),
                           0, s, n, A, lda, j, kend);
    }
    const int64_t rest = n - kend;
    if (rest > 0) {
      hipError_t e = launch_trsm_left(TriMode::LN, kb, rest, A + k0 + k0 * lda, lda,
                                      A + k0 + kend * lda, lda, s);
      if (e != hipSuccess) return e;
      e = launch_dgemm(rest, rest, kb, A + kend + k0 * lda, lda, OpA::General,
                       A + k0 + kend * lda, lda, OpB::General, A + kend + kend * lda, lda,
                       Acc::SubtractTrailing, s);
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

hipError_t launch_ipiv_to_perm(int64_t n, const int64_t *ipiv, int64_t *perm, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const size_t lds = n <= kPermLdsMax ? size_t(n) * sizeof(int32_t) : 0;
  hipLaunchKernelGGL(k_ipiv_to_perm, dim3(1), dim3(64), lds, s, n, ipiv, perm);
  return hipGetLastError();
}

hipError_t launch_gather_rows(int64_t n, int64_t nrhs, const int64_t *perm, const double *B,
                              int64_t ldb, double *Y, int64_t ldy, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  const dim3 grid(unsigned((n + TPB - 1) / TPB), unsigned(nrhs < 65535 ? nrhs : 65535));
  hipLaunchKernelGGL(k_gather_rows, grid, dim3(TPB), 0, s, n, nrhs, perm, B, ldb, Y, ldy);
  return hipGetLastError();
}

}  // namespace rbt
