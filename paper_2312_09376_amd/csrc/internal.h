// Internal declarations shared by the HIP translation units of librbt.
// Not part of the public ABI (include/rbt.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "rbt.h"

namespace rbt {

#define RBT_HIP_CHECK(expr)                                                     \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) {                                                     \
      rbt::report_hip_error(e_, #expr, __FILE__, __LINE__);                     \
      return RBT_ERR_HIP;                                                       \
    }                                                                           \
  } while (0)

void report_hip_error(hipError_t e, const char *what, const char *file, int line);

// Block size of the elimination (diagonal blocks, panel width).
constexpr int kNB = 128;

// Butterfly geometry: m = 2^d ceil(n / 2^d), q = m / 2^d.
struct Geometry {
  int64_t n, m, q;
  int d;
};
inline Geometry geometry(int64_t n, int d) {
  const int64_t g = int64_t(1) << d;
  const int64_t m = g * ((n + g - 1) / g);
  return Geometry{n, m, m / g, d};
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ---- kernel launchers (each defined next to its kernels) ----

// k_butterfly.hip
hipError_t launch_generate(int64_t n, int d, uint64_t seed, double *U, double *V, hipStream_t s);
hipError_t launch_transform2(const Geometry &g, const double *A, int64_t lda, void *out,
                             int64_t ldo, int out_prec, const double *U, const double *V,
                             hipStream_t s);
hipError_t launch_transform_vec(const Geometry &g, int64_t nrhs, double *B, int64_t ldb,
                                const double *C, int op, hipStream_t s);

// k_gemm.hip : C (M x N) op= A (M x K) * B (K x N), FP64, column-major.
// Triangular modes read a packed block inverse W (ld = kNB): strictly lower
// part = L^-1 without its unit diagonal, upper part = U^-1.
enum class OpA {
  General,     // A(m, k) = A[m + k lda]
  GeneralT,    // A(m, k) = A[k + m lda]       (transposed storage)
  UnitLower,   // unit-lower part of W          (L^-1)
  Upper,       // upper part of W               (U^-1)
  UnitLowerT,  // transpose of the unit-lower   (L^-T)
  UpperT       // transpose of the upper        (U^-T)
};
enum class OpB {
  General,  // B(k, n) = B[k + n ldb]
  Upper     // upper part of W (U^-1)
};
enum class Acc { Overwrite, Subtract };
hipError_t launch_dgemm(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda, OpA opa,
                        const double *B, int64_t ldb, OpB opb, double *C, int64_t ldc, Acc acc,
                        hipStream_t s);

// k_getrf.hip : factor the kb x kb diagonal block in place, write the packed
// inverses to Winv (ld kNB); first exact zero pivot -> *info = gofs + c + 1.
hipError_t launch_diag_lu(int kb, double *A, int64_t lda, double *Winv, int64_t gofs,
                          int32_t *info, hipStream_t s);

// k_solve.hip
int64_t rowabs_chunks(int64_t n);
hipError_t launch_anorm(int64_t n, const double *A, int64_t lda, double *partial, double *out,
                        hipStream_t s);
hipError_t launch_berr(int64_t n, int64_t nrhs, const double *R, int64_t ldr, const double *X,
                       int64_t ldx, const double *B, int64_t ldb, const double *anorm,
                       double *colstat, double *berr, hipStream_t s);
hipError_t launch_axpy_cols(int64_t n, int64_t nrhs, const double *D, int64_t ldd, double *X,
                            int64_t ldx, hipStream_t s);
hipError_t launch_copy_cols(int64_t n, int64_t nrhs, const double *S, int64_t lds, double *D,
                            int64_t ldd, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t v, hipStream_t s);

}  // namespace rbt
