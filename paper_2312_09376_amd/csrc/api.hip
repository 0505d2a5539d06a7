// C ABI entry points (include/rbt.h): argument checks, workspace carving and
// the launch sequence of the method (Eq. 1 and the three steps under it).
#include <cstdio>
#include <cstdlib>

#include "internal.h"

namespace rbt {

void report_hip_error(hipError_t e, const char *what, const char *file, int line) {
  if (std::getenv("RBT_QUIET") == nullptr)
    std::fprintf(stderr, "[rbt] HIP error %d (%s) in %s at %s:%d\n", int(e), hipGetErrorString(e),
                 what, file, line);
}

namespace {

inline int64_t nblocks(int64_t n) { return (n + kNB - 1) / kNB; }

// Workspace layout. The packed block inverses come first so that rbt_genp,
// rbt_getrs and the composite entry points agree on where they live.
struct Layout {
  size_t winv, coef, resid, partial, small, total;
  size_t o_winv, o_coef, o_resid, o_partial, o_small;
};

Layout layout(int64_t n, int64_t nrhs, int d) {
  Layout L{};
  L.winv = align256(size_t(nblocks(n)) * kNB * kNB * sizeof(double));
  L.coef = align256(size_t(2) * n * d * sizeof(double));
  L.resid = align256(size_t(n) * nrhs * sizeof(double));
  L.partial = align256(size_t(rowabs_chunks(n)) * n * sizeof(double));
  L.small = align256((3 * size_t(nrhs) + 8) * sizeof(double)) + 256;
  L.o_winv = 0;
  L.o_coef = L.o_winv + L.winv;
  L.o_resid = L.o_coef + L.coef;
  L.o_partial = L.o_resid + L.resid;
  L.o_small = L.o_partial + L.partial;
  L.total = L.o_small + L.small;
  return L;
}

template <typename T>
T *at(void *base, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Blocked right-looking elimination without pivoting (block kNB):
//   factor A11 (and invert its triangles), L21 = A21 U11^-1,
//   U12 = L11^-1 A12, A22 -= L21 U12.
int genp_fp64(int64_t n, double *A, int64_t lda, int32_t *info, double *winv, hipStream_t s) {
  if (info) RBT_HIP_CHECK(launch_fill_i32(info, 0, s));
  for (int64_t k = 0; k < n; k += kNB) {
    const int kb = int(n - k < kNB ? n - k : kNB);
    double *A11 = A + k + k * lda;
    double *W = winv + (k / kNB) * kNB * kNB;
    RBT_HIP_CHECK(launch_diag_lu(kb, A11, lda, W, k, info, s));
    const int64_t rem = n - k - kb;
    if (rem <= 0) continue;
    double *A21 = A + (k + kb) + k * lda;
    double *A12 = A + k + (k + kb) * lda;
    double *A22 = A + (k + kb) + (k + kb) * lda;
    RBT_HIP_CHECK(launch_dgemm(rem, kb, kb, A21, lda, OpA::General, W, kNB, OpB::Upper, A21, lda,
                               Acc::Overwrite, s));
    RBT_HIP_CHECK(launch_dgemm(kb, rem, kb, W, kNB, OpA::UnitLower, A12, lda, OpB::General, A12,
                               lda, Acc::Overwrite, s));
    RBT_HIP_CHECK(launch_dgemm(rem, rem, kb, A21, lda, OpA::General, A12, lda, OpB::General, A22,
                               lda, Acc::Subtract, s));
  }
  return 0;
}

// B <- (LU)^-1 B (trans = 0) or (LU)^-T B (trans = 1), by block solves with
// the packed diagonal-block inverses and GEMM updates.
int getrs_fp64(int64_t n, int64_t nrhs, const double *LU, int64_t ld, double *B, int64_t ldb,
               int trans, const double *winv, hipStream_t s) {
  if (n == 0 || nrhs == 0) return 0;
  const int64_t nb = nblocks(n);
  auto kb_of = [&](int64_t blk) { return int(n - blk * kNB < kNB ? n - blk * kNB : kNB); };
  if (trans == 0) {
    for (int64_t blk = 0; blk < nb; ++blk) {  // L Y = B
      const int64_t k = blk * kNB;
      const int kb = kb_of(blk);
      const double *W = winv + blk * kNB * kNB;
      RBT_HIP_CHECK(launch_dgemm(kb, nrhs, kb, W, kNB, OpA::UnitLower, B + k, ldb, OpB::General,
                                 B + k, ldb, Acc::Overwrite, s));
      const int64_t rem = n - k - kb;
      if (rem > 0)
        RBT_HIP_CHECK(launch_dgemm(rem, nrhs, kb, LU + (k + kb) + k * ld, ld, OpA::General, B + k,
                                   ldb, OpB::General, B + k + kb, ldb, Acc::Subtract, s));
    }
    for (int64_t blk = nb - 1; blk >= 0; --blk) {  // U X = Y
      const int64_t k = blk * kNB;
      const int kb = kb_of(blk);
      const double *W = winv + blk * kNB * kNB;
      RBT_HIP_CHECK(launch_dgemm(kb, nrhs, kb, W, kNB, OpA::Upper, B + k, ldb, OpB::General,
                                 B + k, ldb, Acc::Overwrite, s));
      if (k > 0)
        RBT_HIP_CHECK(launch_dgemm(k, nrhs, kb, LU + k * ld, ld, OpA::General, B + k, ldb,
                                   OpB::General, B, ldb, Acc::Subtract, s));
    }
  } else {
    for (int64_t blk = 0; blk < nb; ++blk) {  // U^T Z = B
      const int64_t k = blk * kNB;
      const int kb = kb_of(blk);
      const double *W = winv + blk * kNB * kNB;
      RBT_HIP_CHECK(launch_dgemm(kb, nrhs, kb, W, kNB, OpA::UpperT, B + k, ldb, OpB::General,
                                 B + k, ldb, Acc::Overwrite, s));
      const int64_t rem = n - k - kb;
      if (rem > 0)
        RBT_HIP_CHECK(launch_dgemm(rem, nrhs, kb, LU + k + (k + kb) * ld, ld, OpA::GeneralT,
                                   B + k, ldb, OpB::General, B + k + kb, ldb, Acc::Subtract, s));
    }
    for (int64_t blk = nb - 1; blk >= 0; --blk) {  // L^T W = Z
      const int64_t k = blk * kNB;
      const int kb = kb_of(blk);
      const double *W = winv + blk * kNB * kNB;
      RBT_HIP_CHECK(launch_dgemm(kb, nrhs, kb, W, kNB, OpA::UnitLowerT, B + k, ldb, OpB::General,
                                 B + k, ldb, Acc::Overwrite, s));
      if (k > 0)
        RBT_HIP_CHECK(launch_dgemm(k, nrhs, kb, LU + k, ld, OpA::GeneralT, B + k, ldb,
                                   OpB::General, B, ldb, Acc::Subtract, s));
    }
  }
  return 0;
}

bool bad_depth(int d) { return d < 0 || d > RBT_MAX_DEPTH; }

}  // namespace
}  // namespace rbt

using namespace rbt;

extern "C" size_t rbt_workspace_size(int64_t n, int64_t nrhs, int depth, int precision) {
  if (n < 0 || nrhs < 0 || bad_depth(depth) || precision != RBT_FP64) return 0;
  return layout(n, nrhs, depth).total;
}

extern "C" int rbt_generate_device(int64_t n, int depth, uint64_t seed, double *dU, double *dV,
                                   void *stream) {
  if (n < 0) return -1;
  if (bad_depth(depth)) return -2;
  if (n > 0 && depth > 0 && dU == nullptr) return -4;
  if (n > 0 && depth > 0 && dV == nullptr) return -5;
  RBT_HIP_CHECK(launch_generate(n, depth, seed, dU, dV, S(stream)));
  return 0;
}

extern "C" int rbt_transform2(int64_t n, const double *A, int64_t lda, void *Out, int64_t ldo,
                              int out_prec, const double *dU, const double *dV, int depth,
                              void *stream) {
  if (n < 0) return -1;
  if (n > 0 && A == nullptr) return -2;
  if (lda < (n > 1 ? n : 1)) return -3;
  if (n > 0 && Out == nullptr) return -4;
  if (ldo < (n > 1 ? n : 1)) return -5;
  if (out_prec != RBT_FP64 && out_prec != RBT_FP32) return -6;
  if (out_prec == RBT_FP64 && (const void *)A == Out && ldo != lda) return -5;
  if (out_prec == RBT_FP32 && depth > 3) return RBT_ERR_UNSUPPORTED;
  if (n > 0 && depth > 0 && dU == nullptr) return -7;
  if (n > 0 && depth > 0 && dV == nullptr) return -8;
  if (bad_depth(depth)) return -9;
  RBT_HIP_CHECK(launch_transform2(geometry(n, depth), A, lda, Out, ldo, out_prec, dU, dV,
                                  S(stream)));
  return 0;
}

extern "C" int rbt_transform_vec(int64_t n, int64_t nrhs, double *B, int64_t ldb, const double *dC,
                                 int depth, int op, void *stream) {
  if (n < 0) return -1;
  if (nrhs < 0) return -2;
  if (n > 0 && nrhs > 0 && B == nullptr) return -3;
  if (ldb < (n > 1 ? n : 1)) return -4;
  if (n > 0 && depth > 0 && dC == nullptr) return -5;
  if (bad_depth(depth)) return -6;
  if (op != RBT_OP_T && op != RBT_OP_N) return -7;
  RBT_HIP_CHECK(launch_transform_vec(geometry(n, depth), nrhs, B, ldb, dC, op, S(stream)));
  return 0;
}

extern "C" int rbt_genp(int64_t n, double *A, int64_t lda, int32_t *info_dev, void *work,
                        size_t work_bytes, void *stream) {
  if (n < 0) return -1;
  if (n > 0 && A == nullptr) return -2;
  if (lda < (n > 1 ? n : 1)) return -3;
  const Layout L = layout(n, 0, 0);
  if (n > 0 && work == nullptr) return -5;
  if (work_bytes < L.winv) return RBT_ERR_WORKSPACE;
  return genp_fp64(n, A, lda, info_dev, at<double>(work, L.o_winv), S(stream));
}

extern "C" int rbt_getrs(int64_t n, int64_t nrhs, const double *LU, int64_t ldlu, double *B,
                         int64_t ldb, int trans, void *work, size_t work_bytes, void *stream) {
  if (n < 0) return -1;
  if (nrhs < 0) return -2;
  if (n > 0 && LU == nullptr) return -3;
  if (ldlu < (n > 1 ? n : 1)) return -4;
  if (n > 0 && nrhs > 0 && B == nullptr) return -5;
  if (ldb < (n > 1 ? n : 1)) return -6;
  if (trans != 0 && trans != 1) return -7;
  const Layout L = layout(n, 0, 0);
  if (n > 0 && work == nullptr) return -8;
  if (work_bytes < L.winv) return RBT_ERR_WORKSPACE;
  return getrs_fp64(n, nrhs, LU, ldlu, B, ldb, trans, at<double>(work, L.o_winv), S(stream));
}

extern "C" int rbt_solve_ex(int64_t n, int64_t nrhs, double *A, int64_t lda, double *B, int64_t ldb,
                            int depth, uint64_t seed, int32_t *info_dev, void *work,
                            size_t work_bytes, void *stream) {
  if (n < 0) return -1;
  if (nrhs < 0) return -2;
  if (n > 0 && A == nullptr) return -3;
  if (lda < (n > 1 ? n : 1)) return -4;
  if (n > 0 && nrhs > 0 && B == nullptr) return -5;
  if (ldb < (n > 1 ? n : 1)) return -6;
  if (bad_depth(depth)) return -7;
  const Layout L = layout(n, nrhs, depth);
  if (n > 0 && work == nullptr) return -10;
  if (work_bytes < L.total) return RBT_ERR_WORKSPACE;
  if (n == 0) return 0;
  hipStream_t s = S(stream);
  const Geometry g = geometry(n, depth);
  double *U = at<double>(work, L.o_coef);
  double *V = U + n * depth;
  double *winv = at<double>(work, L.o_winv);
  RBT_HIP_CHECK(launch_generate(n, depth, seed, U, V, s));
  RBT_HIP_CHECK(launch_transform2(g, A, lda, A, lda, RBT_FP64, U, V, s));
  RBT_HIP_CHECK(launch_transform_vec(g, nrhs, B, ldb, U, RBT_OP_T, s));
  int rc = genp_fp64(n, A, lda, info_dev, winv, s);
  if (rc) return rc;
  rc = getrs_fp64(n, nrhs, A, lda, B, ldb, 0, winv, s);
  if (rc) return rc;
  RBT_HIP_CHECK(launch_transform_vec(g, nrhs, B, ldb, V, RBT_OP_N, s));
  return 0;
}

extern "C" int rbt_solve(int64_t n, int64_t nrhs, double *A, int64_t lda, double *B, int64_t ldb,
                         int depth, uint64_t seed, void *stream) {
  if (n < 0 || nrhs < 0 || bad_depth(depth)) return n < 0 ? -1 : (nrhs < 0 ? -2 : -7);
  const size_t bytes = rbt_workspace_size(n, nrhs, depth, RBT_FP64);
  hipStream_t s = S(stream);
  void *work = nullptr;
  RBT_HIP_CHECK(hipMallocAsync(&work, bytes, s));
  const int rc = rbt_solve_ex(n, nrhs, A, lda, B, ldb, depth, seed, nullptr, work, bytes, stream);
  RBT_HIP_CHECK(hipFreeAsync(work, s));
  return rc;
}

extern "C" int rbt_backward_error(int64_t n, int64_t nrhs, const double *A, int64_t lda,
                                  const double *X, int64_t ldx, const double *B, int64_t ldb,
                                  double *berr_dev, void *work, size_t work_bytes, void *stream) {
  if (n < 0) return -1;
  if (nrhs < 0) return -2;
  if (n > 0 && A == nullptr) return -3;
  if (lda < (n > 1 ? n : 1)) return -4;
  if (n > 0 && nrhs > 0 && X == nullptr) return -5;
  if (ldx < (n > 1 ? n : 1)) return -6;
  if (n > 0 && nrhs > 0 && B == nullptr) return -7;
  if (ldb < (n > 1 ? n : 1)) return -8;
  if (berr_dev == nullptr) return -9;
  const Layout L = layout(n, nrhs, 0);
  if (work == nullptr) return -10;
  if (work_bytes < L.total) return RBT_ERR_WORKSPACE;
  hipStream_t s = S(stream);
  double *R = at<double>(work, L.o_resid);
  double *partial = at<double>(work, L.o_partial);
  double *small = at<double>(work, L.o_small);
  if (n == 0 || nrhs == 0) {
    RBT_HIP_CHECK(hipMemsetAsync(berr_dev, 0, sizeof(double), s));
    return 0;
  }
  RBT_HIP_CHECK(launch_anorm(n, A, lda, partial, small, s));
  RBT_HIP_CHECK(launch_copy_cols(n, nrhs, B, ldb, R, n, s));
  RBT_HIP_CHECK(launch_dgemm(n, nrhs, n, A, lda, OpA::General, X, ldx, OpB::General, R, n,
                             Acc::Subtract, s));
  RBT_HIP_CHECK(launch_berr(n, nrhs, R, n, X, ldx, B, ldb, small, small + 8, berr_dev, s));
  return 0;
}

extern "C" int rbt_solve_refine(int64_t n, int64_t nrhs, const double *A, int64_t lda, double *LU,
                                int64_t ldlu, const double *B, int64_t ldb, double *X, int64_t ldx,
                                int depth, uint64_t seed, double tol, int max_iter,
                                int32_t *iters_dev, double *berr_dev, int32_t *info_dev,
                                void *work, size_t work_bytes, void *stream) {
  if (n < 0) return -1;
  if (nrhs < 0) return -2;
  if (n > 0 && A == nullptr) return -3;
  if (lda < (n > 1 ? n : 1)) return -4;
  if (n > 0 && LU == nullptr) return -5;
  if (ldlu < (n > 1 ? n : 1)) return -6;
  if (n > 0 && nrhs > 0 && B == nullptr) return -7;
  if (ldb < (n > 1 ? n : 1)) return -8;
  if (n > 0 && nrhs > 0 && X == nullptr) return -9;
  if (ldx < (n > 1 ? n : 1)) return -10;
  if (bad_depth(depth)) return -11;
  if (!(tol >= 0.0)) return -13;
  if (max_iter < 0) return -14;
  const Layout L = layout(n, nrhs, depth);
  if (n > 0 && work == nullptr) return -18;
  if (work_bytes < L.total) return RBT_ERR_WORKSPACE;
  hipStream_t s = S(stream);
  double *small = at<double>(work, L.o_small);
  double *berr = berr_dev ? berr_dev : small + 1;
  if (n == 0 || nrhs == 0) {
    RBT_HIP_CHECK(hipMemsetAsync(berr, 0, sizeof(double), s));
    if (iters_dev) RBT_HIP_CHECK(hipMemsetAsync(iters_dev, 0, sizeof(int32_t), s));
    return 0;
  }
  const Geometry g = geometry(n, depth);
  double *U = at<double>(work, L.o_coef);
  double *V = U + n * depth;
  double *winv = at<double>(work, L.o_winv);
  double *R = at<double>(work, L.o_resid);
  double *partial = at<double>(work, L.o_partial);
  double *anorm = small;
  double *colstat = small + 8;

  RBT_HIP_CHECK(launch_generate(n, depth, seed, U, V, s));
  RBT_HIP_CHECK(launch_transform2(g, A, lda, LU, ldlu, RBT_FP64, U, V, s));
  int rc = genp_fp64(n, LU, ldlu, info_dev, winv, s);
  if (rc) return rc;
  RBT_HIP_CHECK(launch_copy_cols(n, nrhs, B, ldb, X, ldx, s));
  RBT_HIP_CHECK(launch_transform_vec(g, nrhs, X, ldx, U, RBT_OP_T, s));
  rc = getrs_fp64(n, nrhs, LU, ldlu, X, ldx, 0, winv, s);
  if (rc) return rc;
  RBT_HIP_CHECK(launch_transform_vec(g, nrhs, X, ldx, V, RBT_OP_N, s));
  RBT_HIP_CHECK(launch_anorm(n, A, lda, partial, anorm, s));

  int it = 0;
  for (;;) {
    RBT_HIP_CHECK(launch_copy_cols(n, nrhs, B, ldb, R, n, s));
    RBT_HIP_CHECK(launch_dgemm(n, nrhs, n, A, lda, OpA::General, X, ldx, OpB::General, R, n,
                               Acc::Subtract, s));
    RBT_HIP_CHECK(launch_berr(n, nrhs, R, n, X, ldx, B, ldb, anorm, colstat, berr, s));
    if (it >= max_iter) break;
    double be_host = 0.0;
    RBT_HIP_CHECK(hipMemcpyAsync(&be_host, berr, sizeof(double), hipMemcpyDeviceToHost, s));
    RBT_HIP_CHECK(hipStreamSynchronize(s));
    if (be_host <= tol) break;
    RBT_HIP_CHECK(launch_transform_vec(g, nrhs, R, n, U, RBT_OP_T, s));
    rc = getrs_fp64(n, nrhs, LU, ldlu, R, n, 0, winv, s);
    if (rc) return rc;
    RBT_HIP_CHECK(launch_transform_vec(g, nrhs, R, n, V, RBT_OP_N, s));
    RBT_HIP_CHECK(launch_axpy_cols(n, nrhs, R, n, X, ldx, s));
    ++it;
  }
  if (iters_dev) {
    RBT_HIP_CHECK(hipMemcpyAsync(iters_dev, &it, sizeof(int32_t), hipMemcpyHostToDevice, s));
    RBT_HIP_CHECK(hipStreamSynchronize(s));
  }
  return 0;
}
