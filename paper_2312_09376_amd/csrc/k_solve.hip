// Kernels around the solve: the residual B - A X with the row sums of |A|
// for ||A||_inf fused into the same pass over A, the backward error of
// Eq. 7, the column updates of iterative refinement (Sec. 5) and the
// outer product of the adjoint.
//
// These are HBM-bound (one read of the matrix, a few columns of output), so
// they run as plain FMA kernels with lanes along rows (coalesced column
// runs of the column-major matrix) and the small right-hand-side block in
// LDS; the matrix-core GEMM is kept for wide right-hand sides.
#include "internal.h"

namespace rbt {

namespace {

constexpr int kRows = 256;       // rows per workgroup
constexpr int64_t kChunk = 256;  // columns per split-K chunk of the residual

// partial[(c N + n) M + m] = sum_{k in chunk c} A[m, k] X[k, n];
// ABS: abspart[c M + m] = sum_{k in chunk c} |A[m, k]|.
template <int NMAX, bool ABS>
__global__ void __launch_bounds__(kRows) k_gemv_partial(int64_t M, int N, int64_t K,
                                                        const double *__restrict__ A,
                                                        int64_t lda,
                                                        const double *__restrict__ X,
                                                        int64_t ldx,
                                                        double *__restrict__ partial,
                                                        double *__restrict__ abspart,
                                                        const int32_t *gate) {
  if (gated(gate)) return;
  __shared__ double xs[kChunk][NMAX];
  const int64_t c = blockIdx.y;
  const int64_t k0 = c * kChunk;
  const int kc = int((K - k0) < kChunk ? (K - k0) : kChunk);
  for (int idx = threadIdx.x; idx < kc * NMAX; idx += kRows) {
    const int k = idx / NMAX, n = idx % NMAX;
    xs[k][n] = n < N ? X[(k0 + k) + int64_t(n) * ldx] : 0.0;
  }
  __syncthreads();
  const int64_t m = int64_t(blockIdx.x) * kRows + threadIdx.x;
  if (m >= M) return;
  double acc[NMAX];
#pragma unroll
  for (int n = 0; n < NMAX; ++n) acc[n] = 0.0;
  double s0 = 0.0, s1 = 0.0;
  const double *Ap = A + m + k0 * lda;
  int k = 0;
#pragma unroll 4
  for (; k + 2 <= kc; k += 2) {
    const double a0 = Ap[int64_t(k) * lda];
    const double a1 = Ap[int64_t(k + 1) * lda];
#pragma unroll
    for (int n = 0; n < NMAX; ++n) acc[n] += a0 * xs[k][n] + a1 * xs[k + 1][n];
    if (ABS) {
      s0 += fabs(a0);
      s1 += fabs(a1);
    }
  }
  for (; k < kc; ++k) {
    const double a0 = Ap[int64_t(k) * lda];
#pragma unroll
    for (int n = 0; n < NMAX; ++n) acc[n] += a0 * xs[k][n];
    if (ABS) s0 += fabs(a0);
  }
#pragma unroll
  for (int n = 0; n < NMAX; ++n)
    if (n < N) partial[(c * N + n) * M + m] = acc[n];
  if (ABS) abspart[c * M + m] = s0 + s1;
}

__device__ __forceinline__ double nanmax(double a, double b) {
  // NaN-propagating maximum: a NaN residual must never look converged
  return (b > a || b != b) ? b : a;
}

// Block-wide NaN-propagating max of one value per thread (kRows threads).
__device__ double block_nanmax(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kRows / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = nanmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// R = B - sum_c partial; per workgroup: max_m |R[:, n]|, |X[:, n]|, |B[:, n]|
// and (ABS) max_m sum_c abspart = a block maximum of the row sums of |A|.
// blockstat[(blk * (3 NMAX + 1)) + ...] layout: [3 n + 0..2] per column, then anorm.
template <int NMAX, bool ABS>
__global__ void __launch_bounds__(kRows) k_resid_reduce(
    int64_t M, int N, int64_t chunks, const double *__restrict__ partial,
    const double *__restrict__ abspart, const double *__restrict__ Bm, int64_t ldb,
    const double *__restrict__ X, int64_t ldx, double *__restrict__ R, int64_t ldr,
    double *__restrict__ blockstat, const int32_t *gate) {
  if (gated(gate)) return;
  __shared__ double sh[kRows];
  const int64_t m = int64_t(blockIdx.x) * kRows + threadIdx.x;
  const bool ok = m < M;
  double *bs = blockstat + int64_t(blockIdx.x) * (3 * NMAX + 1);
  for (int n = 0; n < N; ++n) {
    double r = 0.0, xv = 0.0, bv = 0.0;
    if (ok) {
      double s = 0.0;
      for (int64_t c = 0; c < chunks; ++c) s += partial[(c * N + n) * M + m];
      bv = Bm[m + int64_t(n) * ldb];
      r = bv - s;
      R[m + int64_t(n) * ldr] = r;
      xv = X[m + int64_t(n) * ldx];
    }
    const double mr = block_nanmax(fabs(r), sh);
    const double mx = block_nanmax(fabs(xv), sh);
    const double mb = block_nanmax(fabs(bv), sh);
    if (threadIdx.x == 0) {
      bs[3 * n] = mr;
      bs[3 * n + 1] = mx;
      bs[3 * n + 2] = mb;
    }
  }
  if (ABS) {
    double s = 0.0;
    if (ok)
      for (int64_t c = 0; c < chunks; ++c) s += abspart[c * M + m];
    const double ma = block_nanmax(s, sh);
    if (threadIdx.x == 0) bs[3 * NMAX] = ma;
  }
}

// Final reduction over workgroups: anorm (if ABS) and the backward error.
template <int NMAX, bool ABS>
__global__ void __launch_bounds__(kRows) k_berr_blocks(int64_t nblk, int N,
                                                       const double *__restrict__ blockstat,
                                                       double *__restrict__ anorm,
                                                       double *__restrict__ berr,
                                                       const int32_t *gate) {
  if (gated(gate)) return;
  __shared__ double sh[kRows];
  const int stride = 3 * NMAX + 1;
  double a;
  if (ABS) {
    double v = 0.0;
    for (int64_t b = threadIdx.x; b < nblk; b += kRows) v = nanmax(v, blockstat[b * stride + 3 * NMAX]);
    a = block_nanmax(v, sh);
    if (threadIdx.x == 0) anorm[0] = a;
  } else {
    a = anorm[0];
  }
  double be = 0.0;
  for (int n = 0; n < N; ++n) {
    double r = 0.0, x = 0.0, bb = 0.0;
    for (int64_t b = threadIdx.x; b < nblk; b += kRows) {
      r = nanmax(r, blockstat[b * stride + 3 * n]);
      x = nanmax(x, blockstat[b * stride + 3 * n + 1]);
      bb = nanmax(bb, blockstat[b * stride + 3 * n + 2]);
    }
    r = block_nanmax(r, sh);
    x = block_nanmax(x, sh);
    bb = block_nanmax(bb, sh);
    be = nanmax(be, r / (a * x + bb));
  }
  if (threadIdx.x == 0) berr[0] = be;
}

// ---- wide right-hand sides (N > 16): GEMM residual, separate norms ----

// partial[c * n + i] = sum_{j in chunk c} |A[i, j]|
__global__ void __launch_bounds__(kRows) k_rowabs_partial(int64_t n, const double *__restrict__ A,
                                                         int64_t lda,
                                                         double *__restrict__ partial) {
  const int64_t i = int64_t(blockIdx.x) * kRows + threadIdx.x;
  if (i >= n) return;
  const int64_t j0 = int64_t(blockIdx.y) * kChunk;
  const int64_t j1 = j0 + kChunk < n ? j0 + kChunk : n;
  double s0 = 0.0, s1 = 0.0;
  int64_t j = j0;
  for (; j + 2 <= j1; j += 2) {
    s0 += fabs(A[i + j * lda]);
    s1 += fabs(A[i + (j + 1) * lda]);
  }
  for (; j < j1; ++j) s0 += fabs(A[i + j * lda]);
  partial[int64_t(blockIdx.y) * n + i] = s0 + s1;
}

// blockstat[blk] = max over the block's rows of sum_c partial
__global__ void __launch_bounds__(kRows) k_rowabs_reduce(int64_t n, int64_t chunks,
                                                        const double *__restrict__ partial,
                                                        double *__restrict__ blockstat) {
  __shared__ double sh[kRows];
  const int64_t i = int64_t(blockIdx.x) * kRows + threadIdx.x;
  double s = 0.0;
  if (i < n)
    for (int64_t c = 0; c < chunks; ++c) s += partial[c * n + i];
  const double m = block_nanmax(s, sh);
  if (threadIdx.x == 0) blockstat[blockIdx.x] = m;
}

__global__ void __launch_bounds__(kRows) k_max_reduce(int64_t nblk, const double *__restrict__ v,
                                                     double *__restrict__ out) {
  __shared__ double sh[kRows];
  double m = 0.0;
  for (int64_t b = threadIdx.x; b < nblk; b += kRows) m = nanmax(m, v[b]);
  m = block_nanmax(m, sh);
  if (threadIdx.x == 0) out[0] = m;
}

// colstat[3 c + {0,1,2}] = max |R[:, c]|, max |X[:, c]|, max |B[:, c]|
__global__ void __launch_bounds__(kRows) k_colmax(int64_t n, const double *__restrict__ R,
                                                 int64_t ldr, const double *__restrict__ X,
                                                 int64_t ldx, const double *__restrict__ B,
                                                 int64_t ldb, double *__restrict__ colstat) {
  __shared__ double sh[kRows];
  const int64_t c = blockIdx.x;
  double mr = 0.0, mx = 0.0, mb = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kRows) {
    mr = nanmax(mr, fabs(R[i + c * ldr]));
    mx = nanmax(mx, fabs(X[i + c * ldx]));
    mb = nanmax(mb, fabs(B[i + c * ldb]));
  }
  mr = block_nanmax(mr, sh);
  mx = block_nanmax(mx, sh);
  mb = block_nanmax(mb, sh);
  if (threadIdx.x == 0) {
    colstat[3 * c] = mr;
    colstat[3 * c + 1] = mx;
    colstat[3 * c + 2] = mb;
  }
}

// berr = max_c colstat_r / (anorm * colstat_x + colstat_b)   (Eq. 7 per column)
__global__ void k_berr_final(int64_t nrhs, const double *__restrict__ colstat,
                             const double *__restrict__ anorm, double *__restrict__ berr) {
  if (threadIdx.x != 0) return;
  const double a = anorm[0];
  double m = 0.0;
  for (int64_t c = 0; c < nrhs; ++c)
    m = nanmax(m, colstat[3 * c] / (a * colstat[3 * c + 1] + colstat[3 * c + 2]));
  berr[0] = m;
}

__global__ void __launch_bounds__(kRows) k_axpy_cols(int64_t n, int64_t nrhs,
                                                    const double *__restrict__ D, int64_t ldd,
                                                    double *__restrict__ X, int64_t ldx,
                                                    const int32_t *gate) {
  if (gated(gate)) return;
  const int64_t i = int64_t(blockIdx.x) * kRows + threadIdx.x;
  if (i >= n) return;
  for (int64_t c = blockIdx.y; c < nrhs; c += gridDim.y) X[i + c * ldx] += D[i + c * ldd];
}

__global__ void __launch_bounds__(kRows) k_copy_cols(int64_t n, int64_t nrhs,
                                                    const double *__restrict__ S, int64_t lds,
                                                    double *__restrict__ D, int64_t ldd) {
  const int64_t i = int64_t(blockIdx.x) * kRows + threadIdx.x;
  if (i >= n) return;
  for (int64_t c = blockIdx.y; c < nrhs; c += gridDim.y) D[i + c * ldd] = S[i + c * lds];
}

// dA = -L X^T (n x n, rank nrhs), bound by the n^2 writes: a lane owns two
// consecutive rows of 16 columns, so every store instruction writes 1 KB of
// one column per wavefront (16-byte stores; the operands are only 8-byte
// aligned in general, which these stores accept), and the stores are
// non-temporal (dA is written once and not read back here, so it should not
// displace cached data). The X entries of a column chunk are the same for
// every lane (scalar loads). Each element sums l_k x_k in the order
// k = 0..nrhs-1.
typedef double d2s __attribute__((ext_vector_type(2), aligned(8)));
__global__ void __launch_bounds__(kRows) k_neg_outer(int64_t n, int64_t nrhs,
                                                    const double *__restrict__ Lm, int64_t ldl,
                                                    const double *__restrict__ X, int64_t ldx,
                                                    double *__restrict__ dA, int64_t ldda) {
  const int64_t i = (int64_t(blockIdx.x) * kRows + threadIdx.x) * 2;
  if (i >= n) return;
  const bool pair = i + 1 < n;
  for (int64_t j0 = int64_t(blockIdx.y) * 16; j0 < n; j0 += int64_t(gridDim.y) * 16) {
    double a0[16], a1[16];
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) a0[jj] = a1[jj] = 0.0;
    for (int64_t k = 0; k < nrhs; ++k) {
      const double l0 = Lm[i + k * ldl];
      const double l1 = pair ? Lm[i + 1 + k * ldl] : 0.0;
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        const int64_t j = j0 + jj;
        const double x = (j < n) ? X[j + k * ldx] : 0.0;
        a0[jj] += l0 * x;
        a1[jj] += l1 * x;
      }
    }
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      const int64_t j = j0 + jj;
      if (j >= n) break;
      double *p = dA + i + j * ldda;
      if (pair) {
        const d2s v = {-a0[jj], -a1[jj]};
        __builtin_nontemporal_store(v, reinterpret_cast<d2s *>(p));
      } else {
        __builtin_nontemporal_store(-a0[jj], p);
      }
    }
  }
}

// out[i] = sum_k |A[k, i]| (column sums: ||A||_1 = ||A^T||_inf), one
// workgroup per column.
__global__ void __launch_bounds__(kRows) k_colabs(int64_t n, const double *__restrict__ A,
                                                 int64_t lda, double *__restrict__ out) {
  __shared__ double sh[kRows];
  const int64_t i = blockIdx.x;
  double acc = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += kRows) acc += fabs(A[k + i * lda]);
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int st = kRows / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = sh[0];
}

// Transposed residual R = G - A^T L for N <= NMAX right-hand sides, with
// the column sums of |A| (||A^T||_inf = ||A||_1) fused when ABS. A
// workgroup owns tcols<NMAX>() columns of A (a quarter per wavefront) and
// walks the rows in chunks of kRows: the chunk of L is staged in LDS and
// reused by every column, each wavefront reads its columns of A as
// coalesced runs, and the dot products are reduced across the wavefront at
// the end. A is read once.
template <int NMAX>
constexpr int tcols() {
  return NMAX >= 16 ? 8 : 16;
}
template <int NMAX, bool ABS>
__global__ void __launch_bounds__(kRows) k_gemvT_sub(int64_t n, int N, const double *__restrict__ A,
                                                     int64_t lda, const double *__restrict__ L,
                                                     int64_t ldl, const double *__restrict__ G,
                                                     int64_t ldg, double *__restrict__ R,
                                                     int64_t ldr, double *__restrict__ colabs) {
  constexpr int CW = tcols<NMAX>() / 4;  // columns per wavefront
  __shared__ double Ls[kRows][NMAX];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t j0 = int64_t(blockIdx.x) * tcols<NMAX>() + wave * CW;
  double acc[CW][NMAX];
  double aab[CW];
#pragma unroll
  for (int q = 0; q < CW; ++q) {
    aab[q] = 0.0;
#pragma unroll
    for (int c = 0; c < NMAX; ++c) acc[q][c] = 0.0;
  }
  for (int64_t i0 = 0; i0 < n; i0 += kRows) {
    __syncthreads();
    {
      const int64_t i = i0 + threadIdx.x;
#pragma unroll
      for (int c = 0; c < NMAX; ++c)
        Ls[threadIdx.x][c] = (i < n && c < N) ? L[i + int64_t(c) * ldl] : 0.0;
    }
    __syncthreads();
#pragma unroll 2
    for (int u = 0; u < kRows / 64; ++u) {
      const int r = lane + 64 * u;
      const int64_t i = i0 + r;
      const bool rin = i < n;
#pragma unroll
      for (int q = 0; q < CW; ++q) {
        const int64_t j = j0 + q;
        // clamped, unconditional load; masked by rin / the column bound
        const int64_t jc = j < n ? j : n - 1;
        const double a0 = A[(rin ? i : n - 1) + jc * lda];
        const double a = (rin && j < n) ? a0 : 0.0;
        if constexpr (ABS) aab[q] += fabs(a);
#pragma unroll
        for (int c = 0; c < NMAX; ++c) acc[q][c] += a * Ls[r][c];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < CW; ++q) {
#pragma unroll
    for (int c = 0; c < NMAX; ++c) {
      double v = acc[q][c];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      acc[q][c] = v;
    }
    if constexpr (ABS) {
      double v = aab[q];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      aab[q] = v;
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < CW; ++q) {
      const int64_t j = j0 + q;
      if (j >= n) continue;
#pragma unroll
      for (int c = 0; c < NMAX; ++c)
        if (c < N) R[j + int64_t(c) * ldr] = G[j + int64_t(c) * ldg] - acc[q][c];
      if constexpr (ABS) colabs[j] = aab[q];
    }
  }
}

__global__ void k_refine_step(const double *__restrict__ berr, double tol, int32_t *gate,
                              int32_t *iters) {
  if (threadIdx.x != 0 || *gate != 0) return;
  if (*berr <= tol)  // a NaN error never stops the steps
    *gate = 1;
  else
    *iters += 1;
}

__global__ void k_fill_i32(int32_t *p, int32_t v) {
  if (threadIdx.x == 0) p[0] = v;
}

__global__ void k_fill_f64(double *p, double v) {
  if (threadIdx.x == 0) p[0] = v;
}

// Y[m, n] = sum over split-K chunks of partial (the product A X of
// k_gemv_partial without the residual).
template <int NMAX>
__global__ void __launch_bounds__(kRows) k_gemv_sum(int64_t M, int N, int64_t chunks,
                                                    const double *__restrict__ partial,
                                                    double *__restrict__ Y, int64_t ldy) {
  const int64_t m = int64_t(blockIdx.x) * kRows + threadIdx.x;
  if (m >= M) return;
  for (int n = 0; n < N; ++n) {
    double s = 0.0;
    for (int64_t c = 0; c < chunks; ++c) s += partial[(c * N + n) * M + m];
    Y[m + int64_t(n) * ldy] = s;
  }
}

// Krylov vector kernels (GMRES in FP64 on column blocks of <= kSkinnyMax
// independent columns; basis vector i of column c at V[i * vs + c * n + m]).
// out[i * N + c] = <V_i[:, c], W[:, c]>, one workgroup per (i, c).
__global__ void __launch_bounds__(kRows) k_coldots(int64_t n, int N, const double *__restrict__ V,
                                                   int64_t vs, const double *__restrict__ W,
                                                   int64_t ldw, double *__restrict__ out) {
  __shared__ double sh[kRows];
  const int i = blockIdx.x, c = blockIdx.y;
  const double *v = V + int64_t(i) * vs + int64_t(c) * n;
  const double *w = W + int64_t(c) * ldw;
  double acc = 0.0;
  for (int64_t m = threadIdx.x; m < n; m += kRows) acc += v[m] * w[m];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int st = kRows / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i * N + c] = sh[0];
}

// W[:, c] += sign * sum_{i < J} coef[i * N + c] V_i[:, c]
__global__ void __launch_bounds__(kRows) k_colcombo(int64_t n, int N, int J,
                                                    const double *__restrict__ V, int64_t vs,
                                                    const double *__restrict__ coef, double sign,
                                                    double *__restrict__ W, int64_t ldw) {
  const int64_t m = int64_t(blockIdx.x) * kRows + threadIdx.x;
  const int c = blockIdx.y;
  if (m >= n) return;
  double acc = 0.0;
  for (int i = 0; i < J; ++i) acc += coef[i * N + c] * V[int64_t(i) * vs + int64_t(c) * n + m];
  W[m + int64_t(c) * ldw] += sign * acc;
}

// O[:, c] = W[:, c] / sqrt(nrm2[c]) (zero when nrm2[c] is not positive:
// a column whose Krylov space is exhausted contributes nothing more).
__global__ void __launch_bounds__(kRows) k_colscale(int64_t n, const double *__restrict__ W,
                                                    int64_t ldw, const double *__restrict__ nrm2,
                                                    double *__restrict__ O) {
  const int64_t m = int64_t(blockIdx.x) * kRows + threadIdx.x;
  const int c = blockIdx.y;
  if (m >= n) return;
  const double q = nrm2[c];
  O[m + int64_t(c) * n] = q > 0.0 ? W[m + int64_t(c) * ldw] / sqrt(q) : 0.0;
}

dim3 col_grid(int64_t n, int64_t nrhs) {
  return dim3(unsigned((n + kRows - 1) / kRows), unsigned(nrhs < 65535 ? nrhs : 65535));
}

template <int NMAX>
hipError_t resid_t(int64_t n, int N, const double *A, int64_t lda, const double *X, int64_t ldx,
                   const double *B, int64_t ldb, double *R, int64_t ldr, bool with_anorm,
                   double *partial, double *abspart, double *blockstat, double *anorm,
                   double *berr, hipStream_t s) {
  const int64_t chunks = (n + kChunk - 1) / kChunk;
  const int64_t nblk = (n + kRows - 1) / kRows;
  const dim3 g2 = dim3(unsigned(nblk), unsigned(chunks));
  if (with_anorm) {
    hipLaunchKernelGGL((k_gemv_partial<NMAX, true>), g2, dim3(kRows), 0, s, n, N, n, A, lda, X, ldx, partial, abspart, refine_gate());
    hipLaunchKernelGGL((k_resid_reduce<NMAX, true>), dim3(unsigned(nblk)), dim3(kRows), 0, s, n, N, chunks, partial, abspart, B, ldb, X, ldx, R, ldr, blockstat, refine_gate());
    hipLaunchKernelGGL((k_berr_blocks<NMAX, true>), dim3(1), dim3(kRows), 0, s, nblk, N, blockstat, anorm, berr, refine_gate());
  } else {
    hipLaunchKernelGGL((k_gemv_partial<NMAX, false>), g2, dim3(kRows), 0, s, n, N, n, A, lda, X, ldx, partial, abspart, refine_gate());
    hipLaunchKernelGGL((k_resid_reduce<NMAX, false>), dim3(unsigned(nblk)), dim3(kRows), 0, s, n, N, chunks, partial, abspart, B, ldb, X, ldx, R, ldr, blockstat, refine_gate());
    hipLaunchKernelGGL((k_berr_blocks<NMAX, false>), dim3(1), dim3(kRows), 0, s, nblk, N, blockstat, anorm, berr, refine_gate());
  }
  return hipGetLastError();
}

}  // namespace

size_t resid_scratch_doubles(int64_t n, int64_t nrhs) {
  const int64_t chunks = (n + kChunk - 1) / kChunk;
  const int64_t nblk = (n + kRows - 1) / kRows;
  const int64_t nn = nrhs < 1 ? 1 : nrhs;
  // partial (chunks * max(nrhs,16) * n) + abspart (chunks * n) + blockstat + colstat
  const int64_t w = nn > kSkinnyMax ? 0 : nn;
  return size_t(chunks) * n * (w + 1) + size_t(nblk) * (3 * kSkinnyMax + 1) + 3 * size_t(nn) + 64;
}

hipError_t launch_residual_berr(int64_t n, int64_t nrhs, const double *A, int64_t lda,
                                const double *X, int64_t ldx, const double *B, int64_t ldb,
                                double *R, int64_t ldr, bool with_anorm, double *scratch,
                                double *anorm, double *berr, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) {
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, berr, 0.0);
    return hipGetLastError();
  }
  const int64_t chunks = (n + kChunk - 1) / kChunk;
  const int64_t nblk = (n + kRows - 1) / kRows;
  if (nrhs <= kSkinnyMax) {
    double *partial = scratch;
    double *abspart = partial + chunks * n * nrhs;
    double *blockstat = abspart + chunks * n;
    const int N = int(nrhs);
    if (N <= 1) return resid_t<1>(n, N, A, lda, X, ldx, B, ldb, R, ldr, with_anorm, partial, abspart, blockstat, anorm, berr, s);
    if (N <= 4) return resid_t<4>(n, N, A, lda, X, ldx, B, ldb, R, ldr, with_anorm, partial, abspart, blockstat, anorm, berr, s);
    if (N <= 8) return resid_t<8>(n, N, A, lda, X, ldx, B, ldb, R, ldr, with_anorm, partial, abspart, blockstat, anorm, berr, s);
    return resid_t<16>(n, N, A, lda, X, ldx, B, ldb, R, ldr, with_anorm, partial, abspart, blockstat, anorm, berr, s);
  }
  // wide: norms by their own pass, residual by the matrix-core GEMM
  double *abspart = scratch;
  double *blockstat = abspart + chunks * n;
  double *colstat = blockstat + nblk * (3 * kSkinnyMax + 1);
  if (with_anorm) {
    hipLaunchKernelGGL(k_rowabs_partial, dim3(unsigned(nblk), unsigned(chunks)), dim3(kRows), 0, s, n, A, lda, abspart);
    hipLaunchKernelGGL(k_rowabs_reduce, dim3(unsigned(nblk)), dim3(kRows), 0, s, n, chunks, abspart, blockstat);
    hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(kRows), 0, s, nblk, blockstat, anorm);
  }
  hipLaunchKernelGGL(k_copy_cols, col_grid(n, nrhs), dim3(kRows), 0, s, n, nrhs, B, ldb, R, ldr);
  hipError_t e = launch_dgemm(n, nrhs, n, A, lda, OpA::General, X, ldx, OpB::General, R, ldr,
                              Acc::Subtract, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_colmax, dim3(unsigned(nrhs)), dim3(kRows), 0, s, n, R, ldr, X, ldx, B, ldb, colstat);
  hipLaunchKernelGGL(k_berr_final, dim3(1), dim3(64), 0, s, nrhs, colstat, anorm, berr);
  return hipGetLastError();
}

hipError_t launch_axpy_cols(int64_t n, int64_t nrhs, const double *D, int64_t ldd, double *X,
                            int64_t ldx, hipStream_t s) {
  if (n == 0 || nrhs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy_cols, col_grid(n, nrhs), dim3(kRows), 0, s, n, nrhs, D, ldd, X, ldx, refine_gate());
  return hipGetLastError();
}

hipError_t launch_copy_cols(int64_t n, int64_t nrhs, const double *S, int64_t lds, double *D,
                            int64_t ldd, hipStream_t s) {
  if (n == 0 || nrhs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_cols, col_grid(n, nrhs), dim3(kRows), 0, s, n, nrhs, S, lds, D, ldd);
  return hipGetLastError();
}

hipError_t launch_neg_outer(int64_t n, int64_t nrhs, const double *Lm, int64_t ldl,
                            const double *X, int64_t ldx, double *dA, int64_t ldda,
                            hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t cols = (n + 15) / 16;
  const int64_t rows2 = (n + 1) / 2;  // two rows per lane
  const dim3 grid(unsigned((rows2 + kRows - 1) / kRows), unsigned(cols < 1024 ? cols : 1024));
  hipLaunchKernelGGL(k_neg_outer, grid, dim3(kRows), 0, s, n, nrhs, Lm, ldl, X, ldx, dA, ldda);
  return hipGetLastError();
}

namespace {
thread_local const int32_t *t_gate = nullptr;
}
const int32_t *refine_gate() { return t_gate; }
RefineGate::RefineGate(const int32_t *gate) : prev(t_gate) { t_gate = gate; }
RefineGate::~RefineGate() { t_gate = prev; }

hipError_t launch_refine_step(const double *berr, double tol, int32_t *gate, int32_t *iters,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_refine_step, dim3(1), dim3(64), 0, s, berr, tol, gate, iters);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_matvec(int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *X,
                         int64_t ldx, double *Y, int64_t ldy, double *scratch, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  if (nrhs > kSkinnyMax) return hipErrorInvalidValue;
  const int64_t chunks = (n + kChunk - 1) / kChunk;
  const int64_t nblk = (n + kRows - 1) / kRows;
  const dim3 g2 = dim3(unsigned(nblk), unsigned(chunks));
  const int N = int(nrhs);
  double *partial = scratch;
#define RBT_MATVEC(NM)                                                                          \
  hipLaunchKernelGGL((k_gemv_partial<NM, false>), g2, dim3(kRows), 0, s, n, N, n, A, lda, X,   \
                     ldx, partial, (double *)nullptr, refine_gate());                                          \
  hipLaunchKernelGGL((k_gemv_sum<NM>), dim3(unsigned(nblk)), dim3(kRows), 0, s, n, N, chunks,   \
                     partial, Y, ldy);
  if (N <= 1) {
    RBT_MATVEC(1)
  } else if (N <= 4) {
    RBT_MATVEC(4)
  } else if (N <= 8) {
    RBT_MATVEC(8)
  } else {
    RBT_MATVEC(16)
  }
#undef RBT_MATVEC
  return hipGetLastError();
}

hipError_t launch_coldots(int64_t n, int N, int J, const double *V, int64_t vs, const double *W,
                          int64_t ldw, double *out, hipStream_t s) {
  if (J <= 0 || N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_coldots, dim3(unsigned(J), unsigned(N)), dim3(kRows), 0, s, n, N, V, vs, W,
                     ldw, out);
  return hipGetLastError();
}

hipError_t launch_colcombo(int64_t n, int N, int J, const double *V, int64_t vs,
                           const double *coef, double sign, double *W, int64_t ldw,
                           hipStream_t s) {
  if (J <= 0 || N <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_colcombo, dim3(unsigned((n + kRows - 1) / kRows), unsigned(N)), dim3(kRows),
                     0, s, n, N, J, V, vs, coef, sign, W, ldw);
  return hipGetLastError();
}

hipError_t launch_colscale(int64_t n, int N, const double *W, int64_t ldw, const double *nrm2,
                           double *O, hipStream_t s) {
  if (N <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_colscale, dim3(unsigned((n + kRows - 1) / kRows), unsigned(N)), dim3(kRows),
                     0, s, n, W, ldw, nrm2, O);
  return hipGetLastError();
}

// R = G - A^T L (the residual of the adjoint system A^T L = G) and its Eq. 7
// backward error with ||A^T||_inf = ||A||_1 (with_anorm: computed here into
// *anorm, else read). scratch: n + 3 nrhs doubles.
hipError_t launch_residual_berr_T(int64_t n, int64_t nrhs, const double *A, int64_t lda,
                                  const double *L, int64_t ldl, const double *G, int64_t ldg,
                                  double *R, int64_t ldr, bool with_anorm, double *scratch,
                                  double *anorm, double *berr, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) {
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, berr, 0.0);
    return hipGetLastError();
  }
  double *colabs = scratch;
  double *colstat = scratch + n;
  if (nrhs <= kSkinnyMax) {
    const int N = int(nrhs);
#define RBT_GEMVT(NM)                                                                          \
  const dim3 g(unsigned((n + tcols<NM>() - 1) / tcols<NM>()));                                \
  if (with_anorm)                                                                              \
    hipLaunchKernelGGL((k_gemvT_sub<NM, true>), g, dim3(kRows), 0, s, n, N, A, lda, L, ldl, G,  \
                       ldg, R, ldr, colabs);                                                   \
  else                                                                                         \
    hipLaunchKernelGGL((k_gemvT_sub<NM, false>), g, dim3(kRows), 0, s, n, N, A, lda, L, ldl, G, \
                       ldg, R, ldr, colabs);
    if (N <= 1) {
      RBT_GEMVT(1)
    } else if (N <= 4) {
      RBT_GEMVT(4)
    } else if (N <= 8) {
      RBT_GEMVT(8)
    } else {
      RBT_GEMVT(16)
    }
#undef RBT_GEMVT
    if (with_anorm)
      hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(kRows), 0, s, n, colabs, anorm);
  } else {
    if (with_anorm) {
      hipLaunchKernelGGL(k_colabs, dim3(unsigned(n)), dim3(kRows), 0, s, n, A, lda, colabs);
      hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(kRows), 0, s, n, colabs, anorm);
    }
    hipLaunchKernelGGL(k_copy_cols, col_grid(n, nrhs), dim3(kRows), 0, s, n, nrhs, G, ldg, R, ldr);
    hipError_t e = launch_dgemm(n, nrhs, n, A, lda, OpA::GeneralT, L, ldl, OpB::General, R, ldr,
                                Acc::Subtract, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_colmax, dim3(unsigned(nrhs)), dim3(kRows), 0, s, n, R, ldr, L, ldl, G, ldg,
                     colstat);
  hipLaunchKernelGGL(k_berr_final, dim3(1), dim3(64), 0, s, nrhs, colstat, anorm, berr);
  return hipGetLastError();
}

}  // namespace rbt
