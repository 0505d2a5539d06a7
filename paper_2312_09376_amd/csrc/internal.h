// Internal declarations shared by the HIP translation units of librbt.
// Not part of the public ABI (include/rbt.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

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

// Refinement gate of the capturable refinement: while a RefineGate is alive
// on the calling thread, the launchers of the kernels of one refinement step
// (residual and backward error, one-sided transforms, persistent sweeps,
// the update of X) pass its device word to those kernels, which return at
// once when the word is nonzero. The word is set on the device when the
// backward error has reached tol, so the remaining steps of a fixed count of
// enqueued steps do nothing and no host test is needed between steps.
const int32_t *refine_gate();
struct RefineGate {
  explicit RefineGate(const int32_t *gate);
  ~RefineGate();
  const int32_t *prev;
};
__device__ __forceinline__ bool gated(const int32_t *gate) {
  return gate != nullptr && __hip_atomic_load(gate, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}
// One step of the device-side convergence test: if *gate is 0, set it to
// (*berr <= tol) and, when the error is still above tol, count the
// correction that follows in *iters.
hipError_t launch_refine_step(const double *berr, double tol, int32_t *gate, int32_t *iters,
                              hipStream_t s);

// Butterfly geometry: reference size m = 2^d g ceil(n / (2^d g)) for the
// granule g (1: the non-tiled size of Sec. 3; a tile size n_b: the tiled
// size; lcm(p, q) n_b: the communication-free size of Eq. 8), q = m / 2^d.
// kind: 0 random diagonals with the butterflies of Eq. 2 (Eq. 3), 1 rotation
// butterflies; sides: 2 (U^T A V), 1 (U^T A, the one-sided RBT).
struct Geometry {
  int64_t n, m, q;
  int d;
  int kind, sides;
};
inline Geometry geometry_g(int64_t n, int d, int64_t granule, int kind = 0, int sides = 2) {
  const int64_t g = (int64_t(1) << d) * granule;
  const int64_t m = g * ((n + g - 1) / g);
  return Geometry{n, m, m >> d, d, kind, sides};
}
// The library's structure options (RBT_OPT_GRANULE, RBT_OPT_BUTTERFLY,
// RBT_OPT_SIDES; api.hip).
int64_t butterfly_granule();
int butterfly_kind();
int butterfly_sides();
inline Geometry geometry(int64_t n, int d) {
  return geometry_g(n, d, butterfly_granule(), butterfly_kind(), butterfly_sides());
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ---- stage timing (api.hip) ----
enum Stage {
  kStageGenerate = 0,  // coefficient draw
  kStageTransform2,    // two-sided transform; work = bytes moved (algorithmic)
  kStageTransformVec,  // one-sided transforms; work = bytes moved
  kStageDiag,          // diagonal-block factor + inverse; work = flops (2/3 kb^3 + 2/3 kb^3)
  kStagePanel,         // L21 / U12 block solves as GEMMs; work = flops
  kStageTrailing,      // trailing update A22 -= L21 U12; work = flops 2 rem^2 kb
  kStageSolve,         // block triangular solves; work = flops
  kStageResidual,      // residual, norms, backward error; work = bytes of A read
  kStagePivoted,       // partial-pivoting factorization (fallback); work = flops 2/3 n^3
  kStageOuter,         // adjoint dA = -Lambda X^T; work = bytes written 8 n^2
  kStageCount
};
struct StageScope {
  StageScope(int stage, hipStream_t s, double work);
  ~StageScope();
  int stage_;
  hipStream_t s_;
  hipEvent_t start_ = nullptr;
};

// ---- kernel launchers (each defined next to its kernels) ----

// k_butterfly.hip
// coefficients of g.kind (diagonal entries, or packed cos/sin of the
// rotation butterflies of the structure (n, q, d))
hipError_t launch_generate(const Geometry &g, uint64_t seed, double *U, double *V, hipStream_t s);
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
// SubtractTrailing computes the same as Subtract; it is a separate kernel
// instance so profilers can tell the trailing update of the elimination
// apart from the small updates of the solves.
enum class Acc { Overwrite, Subtract, SubtractTrailing };
hipError_t launch_dgemm(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda, OpA opa,
                        const double *B, int64_t ldb, OpB opb, double *C, int64_t ldc, Acc acc,
                        hipStream_t s);
// C -= A B (General operands) with 64 x 64 (tile = 64) or 128 x 128 block
// tiles; the results are identical (tuning and tests).
hipError_t launch_dgemm_tiles(int tile, int64_t M, int64_t N, int64_t K, const double *A,
                              int64_t lda, const double *B, int64_t ldb, double *C, int64_t ldc,
                              hipStream_t s);
// C0 -= A0 B0 (M0 x N0) and C1 -= A1 B1 (M1 x N1), General operands, depth K,
// leading dimension ld for all six, in one launch of the 64 x 64 tiles (the
// same results as two launches of launch_dgemm with Acc::Subtract). The two
// C regions must not overlap each other or the other update's operands.
hipError_t launch_dgemm_sub2(int64_t K, int64_t ld, int64_t M0, int64_t N0, const double *A0,
                             const double *B0, double *C0, int64_t M1, int64_t N1,
                             const double *A1, const double *B1, double *C1, hipStream_t s);
// k_sgemm.hip : C -= A B with FP32 storage; bf16: BF16 operands on the matrix
// cores (FP32 accumulation), else FP32 operands. trailing: separate kernel
// instance for the trailing update (same arithmetic).
hipError_t launch_sgemm_sub(int64_t M, int64_t N, int64_t K, const float *A, int64_t lda,
                            const float *B, int64_t ldb, float *C, int64_t ldc, bool bf16,
                            bool trailing, hipStream_t s);
// C -= A B (non-trailing instance) with 64 x 64 (tile = 64) or 128 x 128 block
// tiles; the results are identical (tuning and tests).
hipError_t launch_sgemm_tiles(int tile, int64_t M, int64_t N, int64_t K, const float *A,
                              int64_t lda, const float *B, int64_t ldb, float *C, int64_t ldc,
                              bool bf16, hipStream_t s);

// k_getrf.hip : factor the kb x kb diagonal block in place (kb <= kNB);
// first exact zero pivot -> *info = gofs + c + 1. FP32 blocks are
// eliminated in FP32 arithmetic, or with fp64_arith in FP64 and rounded on
// store (the launchers below take the same switch).
hipError_t launch_diag_lu(int kb, double *A, int64_t lda, int64_t gofs, int32_t *info,
                          hipStream_t s);
hipError_t launch_diag_lu(int kb, float *A, int64_t lda, int64_t gofs, int32_t *info,
                          bool fp64_arith, hipStream_t s);

// k_trsm.hip : triangular solves with a factored diagonal block T (kb <= kNB).
enum class TriMode {
  LN,  // L X = B   (unit lower)
  UN,  // U X = B   (upper)
  UT,  // U^T X = B
  LT   // L^T X = B (unit upper)
};
hipError_t launch_trsm_left(TriMode mode, int kb, int64_t N, const double *T, int64_t ldt,
                            double *B, int64_t ldb, hipStream_t s);
hipError_t launch_trsm_left(TriMode mode, int kb, int64_t N, const float *T, int64_t ldt, float *B,
                            int64_t ldb, bool fp64_arith, hipStream_t s);
// X U = B in place, B: M x kb
hipError_t launch_trsm_right_upper(int kb, int64_t M, const double *T, int64_t ldt, double *B,
                                   int64_t ldb, hipStream_t s);
hipError_t launch_trsm_right_upper(int kb, int64_t M, const float *T, int64_t ldt, float *B,
                                   int64_t ldb, bool fp64_arith, hipStream_t s);
// Both solves of a panel step in one launch: Br (M x kb) <- Br U^-1 and
// Bl (kb x N) <- L^-1 Bl with the factored block T (same ldb for both).
hipError_t launch_panel_trsm(int kb, int64_t M, int64_t N, const double *T, int64_t ldt,
                             double *Br, double *Bl, int64_t ldb, hipStream_t s);
hipError_t launch_panel_trsm(int kb, int64_t M, int64_t N, const float *T, int64_t ldt, float *Br,
                             float *Bl, int64_t ldb, bool fp64_arith, hipStream_t s);
// Inverses of all kNB x kNB diagonal blocks of the factors of an n x n
// elimination: block b's L^-1 at W + b * 2 kNB^2 and U^-1 at
// W + b * 2 kNB^2 + kNB^2 (ld kNB). Needs diag_inv_doubles(n) doubles. The
// arithmetic and storage type is that of W (FP32 inverses of FP32 factors
// for FP32 sweeps, FP64 otherwise).
hipError_t launch_diag_inverses(int64_t n, const double *LU, int64_t ld, double *W,
                                hipStream_t s);
hipError_t launch_diag_inverses(int64_t n, const float *LU, int64_t ld, double *W, hipStream_t s);
hipError_t launch_diag_inverses(int64_t n, const float *LU, int64_t ld, float *W, hipStream_t s);
inline int64_t diag_inv_doubles(int64_t n) { return ((n + kNB - 1) / kNB) * 2 * kNB * kNB; }

// k_solve.hip
constexpr int64_t kSkinnyMax = 16;  // right-hand sides handled by the sweeps and FMA kernels
// k_sweep.hip : triangular sweep with op(A) of the factors for
// nrhs <= kSkinnyMax, using the diagonal-block inverses of
// launch_diag_inverses, as ONE persistent launch (ticket-ordered block rows,
// each block's solution published entry by entry). sync:
// sweep_sync_ints(n) int32 of device scratch: words 0..2 are cleared by each
// launch (word 0: the ticket), word 3 is the sticky error word (set when a
// bounded wait expired; the block's solution is then NaN), which the caller
// clears (kSweepErrWord) and reads back; from word 64 (256 bytes) the
// publication buffer, n x kSkinnyMax doubles, reset by each launch.
// FP64 factors take one refinement step per diagonal block, FP32 factors
// the inverse alone.
inline int64_t sweep_sync_ints(int64_t n) { return 64 + 2 * kSkinnyMax * n; }
constexpr int kSweepErrWord = 3;
// Sleeps a sweep's wait may take before it expires (rbt_set_option
// RBT_OPT_SWEEP_SPIN_LIMIT; negative: every wait expires at once).
int64_t sweep_spin_limit();
hipError_t launch_sweep(TriMode mode, int64_t n, int64_t nrhs, const double *LU, int64_t ld,
                        const double *Winv, double *B, int64_t ldb, int32_t *sync, hipStream_t s);
hipError_t launch_sweep(TriMode mode, int64_t n, int64_t nrhs, const float *LU, int64_t ld,
                        const double *Winv, double *B, int64_t ldb, int32_t *sync, hipStream_t s);
// FP32 arithmetic with FP32 inverses (B stays FP64 storage)
hipError_t launch_sweep(TriMode mode, int64_t n, int64_t nrhs, const float *LU, int64_t ld,
                        const float *Winv, double *B, int64_t ldb, int32_t *sync, hipStream_t s);
// doubles of scratch needed by launch_residual_berr
size_t resid_scratch_doubles(int64_t n, int64_t nrhs);
// R = B - A X; berr = Eq. 7 (max over columns); with_anorm: also ||A||_inf -> *anorm
// (otherwise *anorm is read)
hipError_t launch_residual_berr(int64_t n, int64_t nrhs, const double *A, int64_t lda,
                                const double *X, int64_t ldx, const double *B, int64_t ldb,
                                double *R, int64_t ldr, bool with_anorm, double *scratch,
                                double *anorm, double *berr, hipStream_t s);
// Y = A X (n x nrhs, nrhs <= kSkinnyMax); scratch as launch_residual_berr.
hipError_t launch_matvec(int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *X,
                         int64_t ldx, double *Y, int64_t ldy, double *scratch, hipStream_t s);
// Krylov vector operations on N <= kSkinnyMax independent columns; basis
// vector i, column c at V[i * vs + c * n + m].
// out[i * N + c] = <V_i[:, c], W[:, c]> for i < J
hipError_t launch_coldots(int64_t n, int N, int J, const double *V, int64_t vs, const double *W,
                          int64_t ldw, double *out, hipStream_t s);
// W[:, c] += sign * sum_{i < J} coef[i * N + c] V_i[:, c]
hipError_t launch_colcombo(int64_t n, int N, int J, const double *V, int64_t vs,
                           const double *coef, double sign, double *W, int64_t ldw, hipStream_t s);
// O[:, c] (ld n) = W[:, c] / sqrt(nrm2[c]), or 0 when nrm2[c] <= 0
hipError_t launch_colscale(int64_t n, int N, const double *W, int64_t ldw, const double *nrm2,
                           double *O, hipStream_t s);
// R = G - A^T L and the Eq. 7 backward error of the adjoint system
// (||A^T||_inf = ||A||_1); scratch: n + 3 nrhs doubles.
hipError_t launch_residual_berr_T(int64_t n, int64_t nrhs, const double *A, int64_t lda,
                                  const double *L, int64_t ldl, const double *G, int64_t ldg,
                                  double *R, int64_t ldr, bool with_anorm, double *scratch,
                                  double *anorm, double *berr, hipStream_t s);
hipError_t launch_axpy_cols(int64_t n, int64_t nrhs, const double *D, int64_t ldd, double *X,
                            int64_t ldx, hipStream_t s);
hipError_t launch_copy_cols(int64_t n, int64_t nrhs, const double *S, int64_t lds, double *D,
                            int64_t ldd, hipStream_t s);
// dA = -L X^T (n x n) for L, X of n x nrhs
hipError_t launch_neg_outer(int64_t n, int64_t nrhs, const double *Lm, int64_t ldl,
                            const double *X, int64_t ldx, double *dA, int64_t ldda,
                            hipStream_t s);
// k_batched.hip : batched solves in one persistent launch. The host plan
// writes a BatchHeader and `batch` BatchDesc entries (largest systems first)
// into the workspace; the kernel takes entries from the queue in that order.
struct BatchHeader {
  int32_t ticket;  // queue position (reset by each launch)
  int32_t pad0;
  int64_t batch;   // entries in the table
  int32_t depth, prec;
  int64_t f_off_bytes, d_off_bytes, total_bytes;  // FP32 area, FP64 area, workspace used
  int64_t f64_off_bytes;  // FP64 factor area of the fallback (0: none)
};
struct BatchDesc {
  int64_t sys;      // index into the caller's arrays
  int64_t n, nrhs;
  int64_t f_off;    // FP32 factor n x n (ld n), in floats from the FP32 area
  int64_t d_off;    // U, V (n x d each), inverse blocks, residual (n x nrhs), in doubles
  int64_t f64_off;  // FP64 factor n x n (fallback), in doubles from the FP64 factor area
  int64_t pad[2];
};
constexpr size_t kBatchTableOffset = 256;  // descriptors follow the header
// Host part of the plan (batch_plan.cpp, no device calls). Workspace:
// header | descriptor table | FP32 factors | FP64 areas | FP64 fallback
// factors; each system's areas start on 256-byte boundaries.
struct BatchPlanSizes {
  size_t f_off, d_off, f64_off, total;  // byte offsets of the areas; bytes used
};
// 0, or the entry points' error code for negative sizes (-2 n, -3 nrhs) or
// nrhs above kSkinnyMax (RBT_ERR_UNSUPPORTED).
int check_batch_sizes(int64_t batch, const int64_t *n, const int64_t *nrhs);
// Layout for checked sizes; with desc, also the queue: largest systems first,
// systems without work (n = 0 or nrhs = 0) last.
BatchPlanSizes batch_plan_sizes(int64_t batch, const int64_t *n, const int64_t *nrhs, int depth,
                                std::vector<BatchDesc> *desc);
// The bytes rbt_batched_plan copies to the start of the workspace: header
// (ticket 0) and descriptor table.
std::vector<char> batch_plan_image(int64_t batch, int depth, int prec, const BatchPlanSizes &z,
                                   const std::vector<BatchDesc> &desc);
// BF16-operand trailing update with operands staged once (k_hgemm.hip):
// C (FP32) -= bf16(L21) bf16(U12); K must be a multiple of 64.
size_t hgemm_stage_bytes(int64_t M, int64_t N, int64_t K);
bool hgemm_supported(int64_t K);
hipError_t launch_hgemm_sub(int64_t M, int64_t N, int64_t K, const float *L21, int64_t ldl,
                            const float *U12, int64_t ldu, float *C, int64_t ldc, void *stage,
                            size_t stage_bytes, hipStream_t s);

hipError_t launch_batched(int64_t batch, void *work, size_t work_bytes, const double *const *A,
                          const int64_t *lda, const double *const *B, const int64_t *ldb,
                          double *const *X, const int64_t *ldx, int depth, uint64_t seed,
                          int prec, double tol, int max_iter, int32_t *iters, double *berr,
                          int32_t *info, int32_t *path, int grid, int64_t ct2_min_n,
                          hipStream_t s);
// FP64 doubles of one batched system's area (U, V, inverse blocks of 64, residual)
inline int64_t batched_sys_doubles(int64_t n, int64_t nrhs, int d) {
  return 2 * n * d + ((n + 63) / 64) * 64 * 64 + n * nrhs;
}

// k_gepp.hip : elimination with partial pivoting (the robust re-solve of the
// Sec. 5 fallback). launch_gepp factors A in place (P A = L U, ipiv 1-based
// as LAPACK's getrf; *info = first zero pivot column, 1-based) using
// gepp_scratch_bytes() of scratch; launch_ipiv_to_perm turns ipiv into
// perm[i] = original row of row i; launch_gather_rows: Y[i, :] = B[perm[i], :].
constexpr int64_t kPermLdsMax = 16384;  // ipiv_to_perm works in LDS up to this n
size_t gepp_scratch_bytes();
hipError_t launch_gepp(int64_t n, double *A, int64_t lda, int64_t *ipiv, int32_t *info,
                       void *scratch, hipStream_t s);
hipError_t launch_ipiv_to_perm(int64_t n, const int64_t *ipiv, int64_t *perm, hipStream_t s);
hipError_t launch_gather_rows(int64_t n, int64_t nrhs, const int64_t *perm, const double *B,
                              int64_t ldb, double *Y, int64_t ldy, hipStream_t s);

hipError_t launch_fill_i32(int32_t *p, int32_t v, hipStream_t s);
hipError_t launch_fill_f64(double *p, double v, hipStream_t s);

}  // namespace rbt
