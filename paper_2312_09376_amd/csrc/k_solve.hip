// Small kernels around the solve: infinity norms and the backward error of
// Eq. 7, column updates for iterative refinement (Sec. 5), fills and copies.
// The residual product B - A X itself runs on the matrix-core GEMM.
#include "internal.h"

namespace rbt {

namespace {

constexpr int kRowsPerBlock = 256;
constexpr int64_t kColChunk = 512;

// partial[chunk * n + i] = sum_{j in chunk} |A[i, j]|
__global__ void __launch_bounds__(256) k_rowabs_partial(int64_t n, const double *__restrict__ A,
                                                        int64_t lda,
                                                        double *__restrict__ partial) {
  const int64_t i = int64_t(blockIdx.x) * kRowsPerBlock + threadIdx.x;
  if (i >= n) return;
  const int64_t j0 = int64_t(blockIdx.y) * kColChunk;
  const int64_t j1 = j0 + kColChunk < n ? j0 + kColChunk : n;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t j = j0;
  for (; j + 4 <= j1; j += 4) {
    s0 += fabs(A[i + j * lda]);
    s1 += fabs(A[i + (j + 1) * lda]);
    s2 += fabs(A[i + (j + 2) * lda]);
    s3 += fabs(A[i + (j + 3) * lda]);
  }
  for (; j < j1; ++j) s0 += fabs(A[i + j * lda]);
  partial[int64_t(blockIdx.y) * n + i] = (s0 + s1) + (s2 + s3);
}

__device__ __forceinline__ double block_max(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// stats[0] = ||A||_inf = max_i sum_c partial[c * n + i]
__global__ void __launch_bounds__(256) k_anorm(int64_t n, int64_t chunks,
                                               const double *__restrict__ partial,
                                               double *__restrict__ out) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    double s = 0.0;
    for (int64_t c = 0; c < chunks; ++c) s += partial[c * n + i];
    m = fmax(m, s);
  }
  m = block_max(m, sh);
  if (threadIdx.x == 0) out[0] = m;
}

// colstat[3 c + {0,1,2}] = max |R[:, c]|, max |X[:, c]|, max |B[:, c]|
__global__ void __launch_bounds__(256) k_colmax(int64_t n, const double *__restrict__ R,
                                                int64_t ldr, const double *__restrict__ X,
                                                int64_t ldx, const double *__restrict__ B,
                                                int64_t ldb, double *__restrict__ colstat) {
  __shared__ double sh[256];
  const int64_t c = blockIdx.x;
  double mr = 0.0, mx = 0.0, mb = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    // NaN-propagating maxima: a NaN residual must not look converged
    const double vr = fabs(R[i + c * ldr]);
    const double vx = fabs(X[i + c * ldx]);
    const double vb = fabs(B[i + c * ldb]);
    mr = (vr > mr || vr != vr) ? vr : mr;
    mx = (vx > mx || vx != vx) ? vx : mx;
    mb = fmax(mb, vb);
  }
  sh[threadIdx.x] = mr;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double a = sh[threadIdx.x], b = sh[threadIdx.x + s];
      sh[threadIdx.x] = (b > a || b != b) ? b : a;
    }
    __syncthreads();
  }
  const double rr = sh[0];
  __syncthreads();
  const double xx = block_max(mx, sh);
  const double bb = block_max(mb, sh);
  if (threadIdx.x == 0) {
    colstat[3 * c] = rr;
    colstat[3 * c + 1] = xx;
    colstat[3 * c + 2] = bb;
  }
}

// berr = max_c colstat_r / (anorm * colstat_x + colstat_b)   (Eq. 7 per column)
__global__ void k_berr_final(int64_t nrhs, const double *__restrict__ colstat,
                             const double *__restrict__ anorm, double *__restrict__ berr) {
  if (threadIdx.x != 0) return;
  const double a = anorm[0];
  double m = 0.0;
  for (int64_t c = 0; c < nrhs; ++c) {
    const double v = colstat[3 * c] / (a * colstat[3 * c + 1] + colstat[3 * c + 2]);
    m = (v > m || v != v) ? v : m;
  }
  berr[0] = m;
}

__global__ void __launch_bounds__(256) k_axpy_cols(int64_t n, int64_t nrhs,
                                                   const double *__restrict__ D, int64_t ldd,
                                                   double *__restrict__ X, int64_t ldx) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  for (int64_t c = blockIdx.y; c < nrhs; c += gridDim.y) X[i + c * ldx] += D[i + c * ldd];
}

__global__ void __launch_bounds__(256) k_copy_cols(int64_t n, int64_t nrhs,
                                                   const double *__restrict__ S, int64_t lds,
                                                   double *__restrict__ D, int64_t ldd) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  for (int64_t c = blockIdx.y; c < nrhs; c += gridDim.y) D[i + c * ldd] = S[i + c * lds];
}

__global__ void k_fill_i32(int32_t *p, int32_t v) {
  if (threadIdx.x == 0) p[0] = v;
}

dim3 col_grid(int64_t n, int64_t nrhs) {
  return dim3(unsigned((n + 255) / 256), unsigned(nrhs < 65535 ? nrhs : 65535));
}

}  // namespace

int64_t rowabs_chunks(int64_t n) { return (n + kColChunk - 1) / kColChunk; }

hipError_t launch_anorm(int64_t n, const double *A, int64_t lda, double *partial, double *out,
                        hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t chunks = rowabs_chunks(n);
  hipLaunchKernelGGL(k_rowabs_partial, dim3(unsigned((n + 255) / 256), unsigned(chunks)),
                     dim3(256), 0, s, n, A, lda, partial);
  hipLaunchKernelGGL(k_anorm, dim3(1), dim3(256), 0, s, n, chunks, partial, out);
  return hipGetLastError();
}

hipError_t launch_berr(int64_t n, int64_t nrhs, const double *R, int64_t ldr, const double *X,
                       int64_t ldx, const double *B, int64_t ldb, const double *anorm,
                       double *colstat, double *berr, hipStream_t s) {
  if (n == 0 || nrhs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_colmax, dim3(unsigned(nrhs)), dim3(256), 0, s, n, R, ldr, X, ldx, B, ldb,
                     colstat);
  hipLaunchKernelGGL(k_berr_final, dim3(1), dim3(64), 0, s, nrhs, colstat, anorm, berr);
  return hipGetLastError();
}

hipError_t launch_axpy_cols(int64_t n, int64_t nrhs, const double *D, int64_t ldd, double *X,
                            int64_t ldx, hipStream_t s) {
  if (n == 0 || nrhs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy_cols, col_grid(n, nrhs), dim3(256), 0, s, n, nrhs, D, ldd, X, ldx);
  return hipGetLastError();
}

hipError_t launch_copy_cols(int64_t n, int64_t nrhs, const double *S, int64_t lds, double *D,
                            int64_t ldd, hipStream_t s) {
  if (n == 0 || nrhs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_cols, col_grid(n, nrhs), dim3(256), 0, s, n, nrhs, S, lds, D, ldd);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

}  // namespace rbt
