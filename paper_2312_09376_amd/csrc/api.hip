// C ABI entry points (include/rbt.h): argument checks, workspace carving and
// the launch sequence of the method (Eq. 1 and the three steps under it).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <functional>
#include <mutex>
#include <vector>

#include "internal.h"

namespace rbt {

void report_hip_error(hipError_t e, const char *what, const char *file, int line) {
  if (std::getenv("RBT_QUIET") == nullptr)
    std::fprintf(stderr, "[rbt] HIP error %d (%s) in %s at %s:%d\n", int(e), hipGetErrorString(e),
                 what, file, line);
}

// ---- stage timing ----
// When enabled, composite entry points bracket each stage with a pair of HIP
// events on the caller's stream; rbt_timing_read waits for them and returns
// per-stage totals. Off by default (no events are recorded). The records
// are guarded by a mutex: calls on several host threads (one stream each)
// may be timed together.
namespace {
struct TimingState {
  std::mutex mu;
  bool on = false;
  uint32_t mask = (1u << kStageCount) - 1;  // stages timed while on (RBT_OPT_TIMING_STAGES)
  struct Rec {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  double work[kStageCount] = {};
  int64_t launches[kStageCount] = {};
};
TimingState &timing() {
  static TimingState t;
  return t;
}
}  // namespace

StageScope::StageScope(int stage, hipStream_t s, double work) : stage_(stage), s_(s) {
  TimingState &t = timing();
  if (!t.on || ((t.mask >> stage) & 1u) == 0) return;
  if (hipEventCreate(&start_) != hipSuccess) {
    start_ = nullptr;
    return;
  }
  hipEventRecord(start_, s_);
  std::lock_guard<std::mutex> lock(t.mu);
  t.work[stage] += work;
  t.launches[stage] += 1;
}

StageScope::~StageScope() {
  if (start_ == nullptr) return;
  hipEvent_t end = nullptr;
  if (hipEventCreate(&end) != hipSuccess) {
    hipEventDestroy(start_);
    return;
  }
  hipEventRecord(end, s_);
  TimingState &t = timing();
  std::lock_guard<std::mutex> lock(t.mu);
  t.recs.push_back({stage_, start_, end});
}

namespace {

inline int64_t nblocks(int64_t n) { return (n + kNB - 1) / kNB; }

// Rows (from the panel's first row down) from which a panel takes the
// recursive order by default: shorter panels have too few tiles in their
// deeper updates to gain (measured: n = 1000 5-9 % and n = 8191 1 % slower
// with recursive halves, n = 20000 1.5 % faster).
constexpr int64_t kHalvesMinRows = 8192;

// Tunable options (rbt_set_option).
struct Options {
  int64_t outer_nb = 2048;  // width of the panel whose trailing update is one GEMM
  // batched: systems with n >= this take two 64-column tiles per round of
  // the low-precision trailing update, the others one (INT64_MAX: one for all)
  int64_t batch_ct2_min_n = INT64_MAX;
  int64_t batch_wgs_per_cu = 2; // batched: persistent workgroups per compute unit
  int64_t lookahead = 0;        // elimination: overlap panels with the trailing update
  int64_t bf16_staged = 1;      // BF16 elimination: staged-operand trailing GEMM
  int64_t sweep_spin_limit = int64_t(1) << 20;  // sleeps before a sweep's wait expires
  int64_t mixed_fp64_inner = 0;  // mixed precision: diagonal blocks, panel and triangular
                                 // solves in FP64 arithmetic (else FP32)
  int64_t granule = 1;           // butterfly structure: reference-size granule
  int64_t kind = 0;              // butterflies: 0 Eq. 3 (random diagonals), 1 rotations
  int64_t sides = 2;             // 2: U^T A V; 1: U^T A (one-sided)
  int64_t capturable = 0;        // refinement without host tests (graph capturable)
  int64_t panel_split = 2;       // panel: 0 one 128-block after another, 1 recursive halves,
                                 // 2 recursive halves for panels of >= kHalvesMinRows rows
};
Options &options() {
  static Options o;
  return o;
}
}  // namespace

int64_t sweep_spin_limit() { return options().sweep_spin_limit; }
int64_t butterfly_granule() { return options().granule; }
int butterfly_kind() { return int(options().kind); }
int butterfly_sides() { return int(options().sides); }

namespace {

// Workspace layout of the composite entry points. The inverses of the
// diagonal blocks (for the few-right-hand-side solves) come first, so that
// rbt_getrs and the composite entry points agree on where they live.
struct Layout {
  size_t winv, sync, coef, resid, partial, krylov, small, total;
  size_t o_winv, o_sync, o_coef, o_resid, o_partial, o_krylov, o_small;
  // partial pivoting (the GEPP re-solve): ipiv and perm (n int64 each), a
  // row-gather buffer (n x nrhs) and the pivot search's partial maxima
  size_t piv, o_piv, ygat, o_ygat, gscr, o_gscr;
  size_t hstage, o_hstage, total_staged;  // BF16: operand staging of the trailing update
};

// GMRES-IR: Krylov basis per restart cycle and the reduction of the
// preconditioned residual that ends a cycle.
constexpr int kGmresRestart = 50;
constexpr double kGmresTau = 1e-10;
// Guarded GMRES-IR: from iteration kGmresStallMin of a cycle on, the
// residual estimate is extrapolated at the rate of the last kGmresStallWin
// iterations; the refinement stops when the extrapolated backward error at
// the end of the budget exceeds tol by more than the margin.
constexpr int kGmresStallMin = 8;
constexpr int kGmresStallWin = 4;
constexpr double kGmresStallMargin = 1e3;

int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }

// doubles of the GMRES work area: basis (restart + 1 blocks of n x 16), W,
// and small per-column arrays (dots, second dots, norms, coefficients)
size_t krylov_doubles(int64_t n) {
  return size_t(kGmresRestart + 2) * n * kSkinnyMax + size_t(4 * (kGmresRestart + 2)) * kSkinnyMax;
}

// mixed: the mixed-precision entry point (GMRES work area; residual scratch
// also for one group of <= 16 columns).
Layout layout(int64_t n, int64_t nrhs, int d, bool mixed = false, bool bf16 = false) {
  Layout L{};
  L.winv = align256(size_t(diag_inv_doubles(n)) * sizeof(double));
  L.sync = align256(size_t(sweep_sync_ints(n)) * sizeof(int32_t));
  L.coef = align256(size_t(2) * n * d * sizeof(double));
  L.resid = align256(size_t(n) * nrhs * sizeof(double));
  size_t part = resid_scratch_doubles(n, nrhs);
  if (mixed) {
    const size_t p16 = resid_scratch_doubles(n, min64(nrhs, kSkinnyMax));
    part = part > p16 ? part : p16;
  }
  L.partial = align256(part * sizeof(double));
  L.krylov = mixed ? align256(krylov_doubles(n) * sizeof(double)) : 0;
  L.small = 512;
  L.piv = align256(size_t(2) * n * sizeof(int64_t));
  L.ygat = align256(size_t(n) * nrhs * sizeof(double));
  L.gscr = gepp_scratch_bytes();
  L.o_winv = 0;
  L.o_sync = L.o_winv + L.winv;
  L.o_coef = L.o_sync + L.sync;
  L.o_resid = L.o_coef + L.coef;
  L.o_partial = L.o_resid + L.resid;
  L.o_krylov = L.o_partial + L.partial;
  L.o_small = L.o_krylov + L.krylov;
  L.o_piv = L.o_small + L.small;
  L.o_ygat = L.o_piv + L.piv;
  L.o_gscr = L.o_ygat + L.ygat;
  L.total = L.o_gscr + L.gscr;
  // BF16 operands of the trailing update at the current panel width (an
  // optional area after the others: without it the elimination rounds the
  // operands tile by tile)
  L.hstage = bf16 ? align256(hgemm_stage_bytes(n, n, options().outer_nb)) : 0;
  L.o_hstage = L.total;
  L.total_staged = L.total + L.hstage;
  return L;
}

// Sticky error word of the persistent sweeps (k_sweep.hip): cleared at the
// start of every entry point that runs sweeps; the entry points that
// synchronize read it back with their other results (RBT_ERR_SYNC when a
// sweep's bounded wait expired; that block's solution is NaN).
hipError_t clear_sweep_err(int32_t *sync, hipStream_t s) {
  return launch_fill_i32(sync + kSweepErrWord, 0, s);
}
int read_sweep_err(const int32_t *sync, hipStream_t s) {
  int32_t e = 0;
  RBT_HIP_CHECK(hipMemcpyAsync(&e, sync + kSweepErrWord, sizeof(e), hipMemcpyDeviceToHost, s));
  RBT_HIP_CHECK(hipStreamSynchronize(s));
  return e != 0 ? RBT_ERR_SYNC : 0;
}

template <typename T>
T *at(void *base, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }


// GEMM C -= A B of the elimination: FP64 on the FP64 matrix cores, or FP32
// storage with FP32 or BF16 operands (FP32 accumulation).
hipError_t gemm_sub(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda,
                    const double *B, int64_t ldb, double *C, int64_t ldc, int /*prec*/,
                    bool trailing, hipStream_t s) {
  return launch_dgemm(M, N, K, A, lda, OpA::General, B, ldb, OpB::General, C, ldc,
                      trailing ? Acc::SubtractTrailing : Acc::Subtract, s);
}
hipError_t gemm_sub(int64_t M, int64_t N, int64_t K, const float *A, int64_t lda, const float *B,
                    int64_t ldb, float *C, int64_t ldc, int prec, bool trailing, hipStream_t s) {
  return launch_sgemm_sub(M, N, K, A, lda, B, ldb, C, ldc, prec == RBT_BF16, trailing, s);
}

// Both updates that follow a diagonal block's solves inside a panel:
// C0 -= A0 B0 (the panel's columns right of the block, rows below it) and
// C1 -= A1 B1 (the block row's columns right of the panel, the panel's rows
// below the block); depth K, leading dimension ld. One launch in FP64.
hipError_t gemm_sub2(int64_t K, int64_t ld, int64_t M0, int64_t N0, const double *A0,
                     const double *B0, double *C0, int64_t M1, int64_t N1, const double *A1,
                     const double *B1, double *C1, int /*prec*/, hipStream_t s) {
  return launch_dgemm_sub2(K, ld, M0, N0, A0, B0, C0, M1, N1, A1, B1, C1, s);
}
hipError_t gemm_sub2(int64_t K, int64_t ld, int64_t M0, int64_t N0, const float *A0,
                     const float *B0, float *C0, int64_t M1, int64_t N1, const float *A1,
                     const float *B1, float *C1, int prec, hipStream_t s) {
  if (M0 > 0 && N0 > 0) {
    const hipError_t e = gemm_sub(M0, N0, K, A0, ld, B0, ld, C0, ld, prec, false, s);
    if (e != hipSuccess) return e;
  }
  if (M1 > 0 && N1 > 0) return gemm_sub(M1, N1, K, A1, ld, B1, ld, C1, ld, prec, false, s);
  return hipSuccess;
}

// Blocked right-looking elimination without pivoting, two levels:
// the matrix is processed in panels of width W (a multiple of kNB); inside a
// panel, kNB-wide steps factor the diagonal block, solve the rows below it
// (L part) and its block row (U part, kNB rows of the panel's block row
// U12 = L11^-1 A12 at a time), and update the rest of the panel and of its
// block row; then the trailing matrix is updated by one GEMM of depth W,
// which keeps the GEMM's read-modify-write of A22 well under the HBM
// bandwidth at matrix-core rate.
// T = double: FP64 throughout. T = float (mixed precision): FP32 storage
// and FP32 arithmetic (diagonal blocks, triangular solves, GEMM updates with
// FP32 (prec RBT_FP32) or BF16 (RBT_BF16) operands), unless the FP64-inner
// option asks for FP64 diagonal blocks and solves.
// Second stream of the elimination's lookahead, one per device, created on
// first use (default priority, non-blocking) and kept until the process
// ends.
hipStream_t aux_stream() {
  static std::mutex mu;
  static std::vector<hipStream_t> per_dev;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (per_dev.size() <= size_t(dev)) per_dev.resize(dev + 1, nullptr);
  if (per_dev[dev] == nullptr &&
      hipStreamCreateWithFlags(&per_dev[dev], hipStreamNonBlocking) != hipSuccess)
    per_dev[dev] = nullptr;
  return per_dev[dev];
}

// Two events of one elimination (created per call, so that concurrent calls
// never share them).
struct EventPair {
  hipEvent_t f = nullptr, b = nullptr;
  bool ok() const { return f != nullptr && b != nullptr; }
  // created only when the lookahead needs them (without it the elimination
  // creates no runtime objects at all)
  explicit EventPair(bool create) {
    if (!create) return;
    if (hipEventCreateWithFlags(&f, hipEventDisableTiming) != hipSuccess) f = nullptr;
    if (hipEventCreateWithFlags(&b, hipEventDisableTiming) != hipSuccess) b = nullptr;
  }
  ~EventPair() {
    if (f) hipEventDestroy(f);
    if (b) hipEventDestroy(b);
  }
};

// Trailing update A22 -= L21 U12: the staged BF16 GEMM when the operands
// are BF16 and the staging area fits, else the tile-by-tile GEMMs.
hipError_t trailing_sub(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda,
                        const double *B, int64_t ldb, double *C, int64_t ldc, int prec,
                        hipStream_t st, void *, size_t) {
  return gemm_sub(M, N, K, A, lda, B, ldb, C, ldc, prec, true, st);
}
hipError_t trailing_sub(int64_t M, int64_t N, int64_t K, const float *A, int64_t lda,
                        const float *B, int64_t ldb, float *C, int64_t ldc, int prec,
                        hipStream_t st, void *stage, size_t stage_bytes) {
  if (prec == RBT_BF16 && options().bf16_staged && stage != nullptr && hgemm_supported(K) &&
      stage_bytes >= hgemm_stage_bytes(M, N, K))
    return launch_hgemm_sub(M, N, K, A, lda, B, ldb, C, ldc, stage, stage_bytes, st);
  return gemm_sub(M, N, K, A, lda, B, ldb, C, ldc, prec, true, st);
}

// Diagonal-block factor and block solves of the elimination: FP64 for FP64
// factors; FP32 arithmetic for FP32 factors unless the FP64-inner option is
// set.
hipError_t diag_lu(int kb, double *A, int64_t lda, int64_t gofs, int32_t *info, hipStream_t s) {
  return launch_diag_lu(kb, A, lda, gofs, info, s);
}
hipError_t diag_lu(int kb, float *A, int64_t lda, int64_t gofs, int32_t *info, hipStream_t s) {
  return launch_diag_lu(kb, A, lda, gofs, info, options().mixed_fp64_inner != 0, s);
}
hipError_t panel_trsm(int kb, int64_t M, int64_t N, const double *T, int64_t ldt, double *Br,
                      double *Bl, int64_t ldb, hipStream_t s) {
  return launch_panel_trsm(kb, M, N, T, ldt, Br, Bl, ldb, s);
}
hipError_t panel_trsm(int kb, int64_t M, int64_t N, const float *T, int64_t ldt, float *Br,
                      float *Bl, int64_t ldb, hipStream_t s) {
  return launch_panel_trsm(kb, M, N, T, ldt, Br, Bl, ldb, options().mixed_fp64_inner != 0, s);
}
hipError_t trsm_left(TriMode mode, int kb, int64_t N, const double *T, int64_t ldt, double *B,
                     int64_t ldb, hipStream_t s) {
  return launch_trsm_left(mode, kb, N, T, ldt, B, ldb, s);
}
hipError_t trsm_left(TriMode mode, int kb, int64_t N, const float *T, int64_t ldt, float *B,
                     int64_t ldb, hipStream_t s) {
  return launch_trsm_left(mode, kb, N, T, ldt, B, ldb, options().mixed_fp64_inner != 0, s);
}

template <typename T>
int genp_impl(int64_t n, T *A, int64_t lda, int32_t *info, int prec, hipStream_t s,
              void *stage = nullptr, size_t stage_bytes = 0) {
  if (info) RBT_HIP_CHECK(launch_fill_i32(info, 0, s));
  const int64_t W = options().outer_nb;
  // ---- factor the panel A[k0:n, k0:k0+w] (on s). The nt columns right of
  // the panel take their block row U12 = L11^-1 A12 here as well, kNB rows
  // at a time: each diagonal block's left solve runs over the panel's
  // columns and those nt together, and the update of the panel's rows below
  // the block joins the panel's own update in one launch (the same
  // operations on every element as solving the block row after the panel,
  // in fewer launches). ----
  const int64_t split = options().panel_split;
  auto halves = [&](int64_t k0) { return split == 1 || (split == 2 && n - k0 >= kHalvesMinRows); };
  // ---- recursive order of the same panel (RBT_OPT_PANEL_SPLIT = 1): the
  // columns [k, k + w) of a panel whose block-row solves reach column e are
  // split into a left part of ceil(blocks / 2) whole 128-blocks and the
  // rest. The left part is factored first (its diagonal blocks' left solves
  // reach column e); then, with depth h = its width, the rows below it are
  // updated in the right part's columns and the right part's rows in the
  // columns beyond it (up to e), in one launch; then the right part. Every
  // element receives the same updates as in the block-by-block order, in
  // fewer and deeper products: the depth-128 updates become depth-h ones
  // (h up to W / 2), which run closer to the matrix cores' rate and read
  // and write the panel's columns fewer times. ----
  std::function<int(int64_t, int64_t, int64_t)> halves_panel =
      [&](int64_t k, int64_t w, int64_t e) -> int {
    if (w <= kNB) {
      const int kb = int(w);
      T *A11 = A + k + k * lda;
      {
        StageScope t(kStageDiag, s, 2.0 / 3.0 * double(kb) * kb * kb);
        RBT_HIP_CHECK(diag_lu(kb, A11, lda, k, info, s));
      }
      const int64_t rows = n - k - kb, cols = e - k - kb;
      StageScope t(kStagePanel, s, double(rows) * kb * kb + double(cols) * kb * kb);
      RBT_HIP_CHECK(panel_trsm(kb, rows, cols, A11, lda, A + (k + kb) + k * lda,
                               A + k + (k + kb) * lda, lda, s));
      return 0;
    }
    const int64_t h = ((w + kNB - 1) / kNB + 1) / 2 * kNB;
    int rc = halves_panel(k, h, e);
    if (rc) return rc;
    const int64_t rows = n - k - h, wr = w - h, beyond = e - k - w;
    {
      StageScope t(kStagePanel, s, 2.0 * double(h) * (double(rows) * wr + double(wr) * beyond));
      RBT_HIP_CHECK(gemm_sub2(h, lda, rows, wr, A + (k + h) + k * lda, A + k + (k + h) * lda,
                              A + (k + h) + (k + h) * lda, wr, beyond, A + (k + h) + k * lda,
                              A + k + (k + w) * lda, A + (k + h) + (k + w) * lda, prec, s));
    }
    return halves_panel(k + h, wr, e);
  };
  // ---- block rows U12 = L11^-1 A12 of the columns [c0, c0 + nc) for the
  // panel rows [k, k + w), in the recursive order above (used by the
  // lookahead's updates, so that they give the same factors as the panel's
  // own block-row solves) ----
  std::function<int(int64_t, int64_t, int64_t, int64_t, hipStream_t)> halves_rows =
      [&](int64_t k, int64_t w, int64_t c0, int64_t nc, hipStream_t st) -> int {
    if (w <= kNB) {
      StageScope t(kStagePanel, st, double(nc) * w * w);
      RBT_HIP_CHECK(trsm_left(TriMode::LN, int(w), nc, A + k + k * lda, lda, A + k + c0 * lda,
                              lda, st));
      return 0;
    }
    const int64_t h = ((w + kNB - 1) / kNB + 1) / 2 * kNB;
    int rc = halves_rows(k, h, c0, nc, st);
    if (rc) return rc;
    {
      StageScope t(kStagePanel, st, 2.0 * double(w - h) * nc * h);
      RBT_HIP_CHECK(gemm_sub(w - h, nc, h, A + (k + h) + k * lda, lda, A + k + c0 * lda, lda,
                             A + (k + h) + c0 * lda, lda, prec, false, st));
    }
    return halves_rows(k + h, w - h, c0, nc, st);
  };
  auto panel = [&](int64_t k0, int64_t w, int64_t nt) -> int {
    if (halves(k0)) return halves_panel(k0, w, k0 + w + nt);
    for (int64_t k = k0; k < k0 + w; k += kNB) {
      const int kb = int(k0 + w - k < kNB ? k0 + w - k : kNB);
      T *A11 = A + k + k * lda;
      {
        StageScope t(kStageDiag, s, 2.0 / 3.0 * double(kb) * kb * kb);
        RBT_HIP_CHECK(diag_lu(kb, A11, lda, k, info, s));
      }
      const int64_t rows = n - k - kb;      // rows below the diagonal block
      const int64_t pc = k0 + w - k - kb;   // panel columns right of it (= panel rows below it)
      {
        StageScope t(kStagePanel, s, double(rows) * kb * kb + double(pc + nt) * kb * kb);
        RBT_HIP_CHECK(panel_trsm(kb, rows, pc + nt, A11, lda, A + (k + kb) + k * lda,
                                        A + k + (k + kb) * lda, lda, s));
      }
      if (pc > 0 && (rows > 0 || nt > 0)) {
        StageScope t(kStagePanel, s, 2.0 * double(kb) * (double(rows) * pc + double(pc) * nt));
        RBT_HIP_CHECK(gemm_sub2(kb, lda, rows, pc, A + (k + kb) + k * lda, A + k + (k + kb) * lda,
                                A + (k + kb) + (k + kb) * lda, pc, nt, A + (k + kb) + k * lda,
                                A + k + (k0 + w) * lda, A + (k + kb) + (k0 + w) * lda, prec, s));
      }
    }
    return 0;
  };
  // ---- columns [c0, c0 + nc) right of the panel [k0, k0 + w): block row
  // U12 = L11^-1 A12 (L11: w x w unit lower, kNB rows at a time; skipped
  // when the panel solved it: rows_done), then A22 -= L21 U12 with one GEMM
  // of depth w (on stream st) ----
  auto update = [&](int64_t k0, int64_t w, int64_t c0, int64_t nc, hipStream_t st,
                    bool rows_done) -> int {
    if (halves(k0) && !rows_done) {
      const int rc = halves_rows(k0, w, c0, nc, st);
      if (rc) return rc;
      rows_done = true;
    }
    for (int64_t k = k0; k < k0 + w && !rows_done; k += kNB) {
      const int kb = int(k0 + w - k < kNB ? k0 + w - k : kNB);
      const int64_t below = k0 + w - k - kb;
      {
        StageScope t(kStagePanel, st, double(nc) * kb * kb);
        RBT_HIP_CHECK(trsm_left(TriMode::LN, kb, nc, A + k + k * lda, lda,
                                       A + k + c0 * lda, lda, st));
      }
      if (below > 0) {
        StageScope t(kStagePanel, st, 2.0 * double(below) * nc * kb);
        RBT_HIP_CHECK(gemm_sub(below, nc, kb, A + (k + kb) + k * lda, lda, A + k + c0 * lda, lda,
                               A + (k + kb) + c0 * lda, lda, prec, false, st));
      }
    }
    const int64_t rows = n - k0 - w;
    StageScope t(kStageTrailing, st, 2.0 * double(rows) * nc * w);
    // the staging area serves one update at a time: not the lookahead's
    RBT_HIP_CHECK(trailing_sub(rows, nc, w, A + (k0 + w) + k0 * lda, lda, A + k0 + c0 * lda, lda,
                               A + (k0 + w) + c0 * lda, lda, prec, st,
                               st == s ? stage : nullptr, stage_bytes));
    return 0;
  };
  // Lookahead: after panel p, stream s updates only the next panel's columns
  // and factors that panel while the second stream updates the remaining
  // columns (the bulk of the flops); s waits for it before the next block
  // row, which reads those columns. The two streams touch disjoint columns
  // and every element sees the same operations in the same order as without
  // lookahead (the split is at a multiple of the GEMM tile), so the factors
  // are identical either way.
  hipStream_t s2 = options().lookahead ? aux_stream() : nullptr;
  EventPair ev(s2 != nullptr);
  if (s2 != nullptr && !ev.ok()) s2 = nullptr;
  if (n <= 0) return 0;
  // The first panel also takes the n mod kNB columns that do not fill a
  // diagonal block, so that every trailing update is a whole number of
  // 128-wide blocks (a partial tile row and column cost the large-tile GEMM
  // as much as whole ones). Not with BF16 updates: their staged GEMM wants
  // a depth that is a multiple of 64.
  const int64_t r0 = prec == RBT_BF16 ? 0 : n % kNB;
  auto width = [&](int64_t k0) {
    const int64_t w = k0 == 0 ? W + r0 : W;
    return n - k0 < w ? n - k0 : w;
  };
  // Without lookahead every panel solves the block rows of all columns to
  // its right; with it the block rows stay in the updates, which the second
  // stream runs while the next panel is factored.
  const bool la = s2 != nullptr;
  auto trailing_cols = [&](int64_t k0, int64_t w) { return la ? int64_t(0) : n - k0 - w; };
  int rc = panel(0, width(0), trailing_cols(0, width(0)));
  if (rc) return rc;
  for (int64_t k0 = 0, w = width(0);; k0 += w, w = width(k0)) {
    const int64_t rest = n - k0 - w;  // columns right of the panel
    if (rest <= 0) break;
    const int64_t wn = width(k0 + w);  // next panel
    const bool split = la && rest > wn;
    if (split) {
      RBT_HIP_CHECK(hipEventRecord(ev.f, s));
      RBT_HIP_CHECK(hipStreamWaitEvent(s2, ev.f, 0));
      rc = update(k0, w, k0 + w + wn, rest - wn, s2, !la);
      if (rc) return rc;
      RBT_HIP_CHECK(hipEventRecord(ev.b, s2));
    }
    rc = update(k0, w, k0 + w, split ? wn : rest, s, !la);
    if (rc) return rc;
    rc = panel(k0 + w, wn, trailing_cols(k0 + w, wn));
    if (rc) return rc;
    if (split) RBT_HIP_CHECK(hipStreamWaitEvent(s, ev.b, 0));
  }
  return 0;
}

int genp_fp64(int64_t n, double *A, int64_t lda, int32_t *info, hipStream_t s) {
  return genp_impl(n, A, lda, info, RBT_FP64, s);
}

// B <- (LU)^-1 B (trans = 0) or (LU)^-T B (trans = 1): block solves with the
// diagonal blocks (k_trsm.hip) and updates of the remaining rows, by the
// FMA kernel for few right-hand sides and the matrix-core GEMM otherwise.
int getrs_fp64(int64_t n, int64_t nrhs, const double *LU, int64_t ld, double *B, int64_t ldb,
               int trans, const double *winv, int32_t *sync, hipStream_t s) {
  if (n == 0 || nrhs == 0) return 0;
  if (nrhs <= kSkinnyMax) {
    // one persistent launch per sweep: inverse + one refinement step per block
    RBT_HIP_CHECK(launch_sweep(trans ? TriMode::UT : TriMode::LN, n, nrhs, LU, ld, winv, B, ldb,
                               sync, s));
    RBT_HIP_CHECK(launch_sweep(trans ? TriMode::LT : TriMode::UN, n, nrhs, LU, ld, winv, B, ldb,
                               sync, s));
    return 0;
  }
  const int64_t nb = nblocks(n);
  auto kb_of = [&](int64_t blk) { return int(n - blk * kNB < kNB ? n - blk * kNB : kNB); };
  // Y (M x nrhs) -= op(A) (M x kb) X (kb x nrhs) on the matrix cores
  auto update = [&](int64_t M, int kb, const double *Ab, bool tr, const double *X,
                    double *Y) -> hipError_t {
    if (M <= 0) return hipSuccess;
    return launch_dgemm(M, nrhs, kb, Ab, ld, tr ? OpA::GeneralT : OpA::General, X, ldb,
                        OpB::General, Y, ldb, Acc::Subtract, s);
  };
  if (trans == 0) {
    for (int64_t blk = 0; blk < nb; ++blk) {  // L Y = B
      const int64_t k = blk * kNB;
      const int kb = kb_of(blk);
      const double *T = LU + k + k * ld;
      RBT_HIP_CHECK(launch_trsm_left(TriMode::LN, kb, nrhs, T, ld, B + k, ldb, s));
      RBT_HIP_CHECK(update(n - k - kb, kb, LU + (k + kb) + k * ld, false, B + k, B + k + kb));
    }
    for (int64_t blk = nb - 1; blk >= 0; --blk) {  // U X = Y
      const int64_t k = blk * kNB;
      const int kb = kb_of(blk);
      const double *T = LU + k + k * ld;
      RBT_HIP_CHECK(launch_trsm_left(TriMode::UN, kb, nrhs, T, ld, B + k, ldb, s));
      RBT_HIP_CHECK(update(k, kb, LU + k * ld, false, B + k, B));
    }
  } else {
    for (int64_t blk = 0; blk < nb; ++blk) {  // U^T Z = B
      const int64_t k = blk * kNB;
      const int kb = kb_of(blk);
      const double *T = LU + k + k * ld;
      RBT_HIP_CHECK(launch_trsm_left(TriMode::UT, kb, nrhs, T, ld, B + k, ldb, s));
      RBT_HIP_CHECK(update(n - k - kb, kb, LU + k + (k + kb) * ld, true, B + k, B + k + kb));
    }
    for (int64_t blk = nb - 1; blk >= 0; --blk) {  // L^T W = Z
      const int64_t k = blk * kNB;
      const int kb = kb_of(blk);
      const double *T = LU + k + k * ld;
      RBT_HIP_CHECK(launch_trsm_left(TriMode::LT, kb, nrhs, T, ld, B + k, ldb, s));
      RBT_HIP_CHECK(update(k, kb, LU + k, true, B + k, B));
    }
  }
  return 0;
}

// Stage-timed wrappers of the launches used by the composite entry points.
hipError_t generate_t(int64_t n, int d, uint64_t seed, double *U, double *V, hipStream_t s) {
  StageScope t(kStageGenerate, s, 16.0 * double(n) * d);
  return launch_generate(geometry(n, d), seed, U, V, s);
}
// x = V x~ (op N) or V^T g (op T): nothing for the one-sided RBT (V = I).
hipError_t transform_v_t(const Geometry &g, int64_t nrhs, double *B, int64_t ldb,
                         const double *V, int op, hipStream_t s);
hipError_t transform2_t(const Geometry &g, const double *A, int64_t lda, void *out, int64_t ldo,
                        int prec, const double *U, const double *V, hipStream_t s) {
  const double elt_out = prec == RBT_FP32 ? 4.0 : 8.0;
  StageScope t(kStageTransform2, s, (8.0 + elt_out) * double(g.n) * g.n);
  return launch_transform2(g, A, lda, out, ldo, prec, U, V, s);
}
hipError_t transform_vec_t(const Geometry &g, int64_t nrhs, double *B, int64_t ldb,
                           const double *C, int op, hipStream_t s) {
  StageScope t(kStageTransformVec, s, 16.0 * double(g.n) * nrhs);
  return launch_transform_vec(g, nrhs, B, ldb, C, op, s);
}
hipError_t transform_v_t(const Geometry &g, int64_t nrhs, double *B, int64_t ldb,
                         const double *V, int op, hipStream_t s) {
  if (g.sides == 1) return hipSuccess;
  return transform_vec_t(g, nrhs, B, ldb, V, op, s);
}
int getrs_t(int64_t n, int64_t nrhs, const double *LU, int64_t ld, double *B, int64_t ldb,
            int trans, const double *winv, int32_t *sync, hipStream_t s) {
  StageScope t(kStageSolve, s, 2.0 * double(n) * n * nrhs);
  return getrs_fp64(n, nrhs, LU, ld, B, ldb, trans, winv, sync, s);
}
// Inverses of the diagonal blocks, needed by the few-right-hand-side solves.
int diag_inverses_t(int64_t n, int64_t nrhs, const double *LU, int64_t ld, double *winv,
                    hipStream_t s) {
  if (nrhs > kSkinnyMax || n == 0) return 0;
  StageScope t(kStageSolve, s, 2.0 / 3.0 * double(n) * kNB * kNB);
  RBT_HIP_CHECK(launch_diag_inverses(n, LU, ld, winv, s));
  return 0;
}

// Mixed precision: inverses of the diagonal blocks of the FP32 factors,
// always formed, since every solve with FP32 factors runs as sweeps: FP32
// inverses (in the first half of the FP64-sized area), or FP64 ones with
// the FP64-inner option.
int diag_inverses_t(int64_t n, const float *LU, int64_t ld, double *winv, bool f64,
                    hipStream_t s) {
  if (n == 0) return 0;
  StageScope t(kStageSolve, s, 2.0 / 3.0 * double(n) * kNB * kNB);
  if (f64)
    RBT_HIP_CHECK(launch_diag_inverses(n, LU, ld, winv, s));
  else
    RBT_HIP_CHECK(launch_diag_inverses(n, LU, ld, reinterpret_cast<float *>(winv), s));
  return 0;
}
// B <- (LU)^-1 B or (LU)^-T B with FP32 factors and FP64 right-hand sides:
// sweeps over groups of at most kSkinnyMax columns, in FP32 arithmetic (the
// right-hand side rounded to FP32 on load, the result widened on store), or
// in FP64 arithmetic (f64: the FP64-inner option, and the preconditioner of
// GMRES-IR, which that method applies in the working precision). The
// inverses must have been formed by diag_inverses_t with the same f64.
int getrs_t(int64_t n, int64_t nrhs, const float *LU, int64_t ld, double *B, int64_t ldb,
            int trans, const double *winv, int32_t *sync, bool f64, hipStream_t s) {
  StageScope t(kStageSolve, s, 2.0 * double(n) * n * nrhs);
  const float *winv32 = reinterpret_cast<const float *>(winv);
  for (int64_t c0 = 0; c0 < nrhs; c0 += kSkinnyMax) {
    const int64_t nc = nrhs - c0 < kSkinnyMax ? nrhs - c0 : kSkinnyMax;
    double *Bc = B + c0 * ldb;
    for (int pass = 0; pass < 2; ++pass) {
      const TriMode m = pass == 0 ? (trans ? TriMode::UT : TriMode::LN)
                                  : (trans ? TriMode::LT : TriMode::UN);
      if (f64)
        RBT_HIP_CHECK(launch_sweep(m, n, nc, LU, ld, winv, Bc, ldb, sync, s));
      else
        RBT_HIP_CHECK(launch_sweep(m, n, nc, LU, ld, winv32, Bc, ldb, sync, s));
    }
  }
  return 0;
}

// R <- V (L U)^-1 U^T R: the solve of Eq. 1 with the factors of A~ (f64:
// arithmetic of the triangular solves with FP32 factors, see getrs_t).
int getrs_t(int64_t n, int64_t nrhs, const double *LU, int64_t ld, double *B, int64_t ldb,
            int trans, const double *winv, int32_t *sync, bool /*f64*/, hipStream_t s) {
  return getrs_t(n, nrhs, LU, ld, B, ldb, trans, winv, sync, s);
}
template <typename TF>
int apply_solve(const Geometry &g, int64_t nrhs, const TF *LU, int64_t ld, double *R, int64_t ldr,
                const double *U, const double *V, const double *winv, int32_t *sync, bool f64,
                hipStream_t s) {
  RBT_HIP_CHECK(transform_vec_t(g, nrhs, R, ldr, U, RBT_OP_T, s));
  const int rc = getrs_t(g.n, nrhs, LU, ld, R, ldr, 0, winv, sync, f64, s);
  if (rc) return rc;
  RBT_HIP_CHECK(transform_v_t(g, nrhs, R, ldr, V, RBT_OP_N, s));
  return 0;
}

// Classical iterative refinement (Sec. 5): R = B - A X in FP64 with the
// original A, Eq. 7 backward error, X += V (LU)^-1 U^T R, until the backward
// error is <= tol or max_iter corrections have been applied. X holds the
// first solution on entry. The host reads the backward error once per
// iteration (one stream synchronization).
template <typename TF>
int refine_classic(int64_t n, int64_t nrhs, const double *A, int64_t lda, const TF *LU,
                   int64_t ldlu, const double *B, int64_t ldb, double *X, int64_t ldx,
                   const Geometry &g, const double *U, const double *V, const double *winv,
                   int32_t *sync, double *R, double *scratch, double *anorm, double *berr, double tol,
                   int max_iter, int *it_out, bool f64, hipStream_t s, bool *stalled = nullptr) {
  int it = 0;
  double be_prev = 0.0;
  for (;;) {
    {
      StageScope t(kStageResidual, s, 8.0 * double(n) * n);
      RBT_HIP_CHECK(launch_residual_berr(n, nrhs, A, lda, X, ldx, B, ldb, R, n, it == 0, scratch,
                                         anorm, berr, s));
    }
    if (it >= max_iter) break;
    double be_host = 0.0;
    RBT_HIP_CHECK(hipMemcpyAsync(&be_host, berr, sizeof(double), hipMemcpyDeviceToHost, s));
    if (const int e = read_sweep_err(sync, s)) return e;  // also waits for be_host
    if (be_host <= tol) break;
    // guarded use: a non-finite error, or a correction that did not halve
    // the error, means these factors cannot reach tol (the caller falls back)
    if (stalled && (!(be_host < HUGE_VAL) || (it > 0 && !(be_host < 0.5 * be_prev)))) {
      *stalled = true;
      break;
    }
    be_prev = be_host;
    const int rc = apply_solve(g, nrhs, LU, ldlu, R, n, U, V, winv, sync, f64, s);
    if (rc) return rc;
    RBT_HIP_CHECK(launch_axpy_cols(n, nrhs, R, n, X, ldx, s));
    ++it;
  }
  *it_out = it;
  return 0;
}

// Capturable form of refine_classic (the same residuals, corrections and
// stopping rule): all max_iter steps are enqueued at once and each step's
// kernels are gated by a device word that the step's convergence test sets
// when the Eq. 7 error is <= tol, so no host test, synchronization or copy
// is needed and the whole refinement can be captured in a HIP graph. The
// step count goes to *iters on the device. Right-hand sides: at most
// kSkinnyMax (the gated sweep path).
template <typename TF>
int refine_classic_device(int64_t n, int64_t nrhs, const double *A, int64_t lda, const TF *LU,
                          int64_t ldlu, const double *B, int64_t ldb, double *X, int64_t ldx,
                          const Geometry &g, const double *U, const double *V,
                          const double *winv, int32_t *sync, double *R, double *scratch,
                          double *anorm, double *berr, double tol, int max_iter, int32_t *gate,
                          int32_t *iters, bool f64, hipStream_t s) {
  RBT_HIP_CHECK(launch_fill_i32(gate, 0, s));
  RBT_HIP_CHECK(launch_fill_i32(iters, 0, s));
  {
    StageScope t(kStageResidual, s, 8.0 * double(n) * n);
    RBT_HIP_CHECK(launch_residual_berr(n, nrhs, A, lda, X, ldx, B, ldb, R, n, true, scratch,
                                       anorm, berr, s));
  }
  RefineGate on(gate);
  for (int it = 0; it < max_iter; ++it) {
    RBT_HIP_CHECK(launch_refine_step(berr, tol, gate, iters, s));
    const int rc = apply_solve(g, nrhs, LU, ldlu, R, n, U, V, winv, sync, f64, s);
    if (rc) return rc;
    RBT_HIP_CHECK(launch_axpy_cols(n, nrhs, R, n, X, ldx, s));
    StageScope t(kStageResidual, s, 8.0 * double(n) * n);
    RBT_HIP_CHECK(launch_residual_berr(n, nrhs, A, lda, X, ldx, B, ldb, R, n, false, scratch,
                                       anorm, berr, s));
  }
  return 0;
}

// GMRES-IR: each refinement step solves A D = R (R = B - A X in FP64 with
// the original A) by restarted GMRES in FP64, left-preconditioned by
// M^-1 = V (LU)^-1 U^T (the solve of Eq. 1 with the low-precision factors),
// and adds D to X. A cycle ends when the preconditioned residual estimate
// of every column has dropped by kGmresTau, or after kGmresRestart
// iterations; the refinement ends when the Eq. 7 backward error is <= tol
// or max_iter Krylov iterations are spent. Columns are processed in groups
// of <= kSkinnyMax with independent Krylov spaces; classical Gram-Schmidt
// with one reorthogonalization; the small Hessenberg least-squares problems
// (Givens rotations) are solved on the host, one synchronization per
// iteration. *it_out = Krylov iterations of the group that needed most.
template <typename TF>
int refine_gmres(int64_t n, int64_t nrhs, const double *A, int64_t lda, const TF *LU,
                 int64_t ldlu, const double *B, int64_t ldb, double *X, int64_t ldx,
                 const Geometry &g, const double *U, const double *V, const double *winv,
                 int32_t *sync, double *R, double *scratch, double *kry, double *anorm,
                 double *berr, double tol, int max_iter, int *it_out, hipStream_t s,
                 bool *stalled = nullptr) {
  const int m = kGmresRestart;
  const int64_t vs = n * kSkinnyMax;  // stride of basis blocks
  double *Vb = kry;
  double *W = Vb + (m + 1) * vs;
  double *dots = W + vs;
  double *dots2 = dots + (m + 2) * kSkinnyMax;
  double *nrm = dots2 + (m + 2) * kSkinnyMax;
  double *coef = nrm + (m + 2) * kSkinnyMax;
  std::vector<double> hd((m + 2) * kSkinnyMax), hd2((m + 2) * kSkinnyMax), hn(kSkinnyMax);
  std::vector<double> H, cs, sn, gv, beta, y, hist;
  std::vector<int> kc;
  std::vector<char> active;
  int worst = 0;
  bool first = true;
  auto residual = [&](int64_t nc, double *Xc, const double *Bc) -> int {
    StageScope t(kStageResidual, s, 8.0 * double(n) * n);
    RBT_HIP_CHECK(launch_residual_berr(n, nc, A, lda, Xc, ldx, Bc, ldb, R, n, first, scratch,
                                       anorm, berr, s));
    first = false;
    return 0;
  };
  for (int64_t c0 = 0; c0 < nrhs; c0 += kSkinnyMax) {
    const int nc = int(min64(kSkinnyMax, nrhs - c0));
    double *Xc = X + c0 * ldx;
    const double *Bc = B + c0 * ldb;
    int total = 0;
    for (;;) {
      int rc = residual(nc, Xc, Bc);
      if (rc) return rc;
      double be = 0.0;
      RBT_HIP_CHECK(hipMemcpyAsync(&be, berr, sizeof(double), hipMemcpyDeviceToHost, s));
      if (const int e = read_sweep_err(sync, s)) return e;  // also waits for be
      if (be <= tol || total >= max_iter) break;
      if (stalled && !(be < HUGE_VAL)) {
        *stalled = true;
        break;
      }
      bool stop = false;
      // z = M^-1 r, v_0 = z / ||z||
      rc = apply_solve(g, nc, LU, ldlu, R, n, U, V, winv, sync, true, s);
      if (rc) return rc;
      RBT_HIP_CHECK(launch_coldots(n, nc, 1, R, 0, R, n, nrm, s));
      RBT_HIP_CHECK(launch_colscale(n, nc, R, n, nrm, Vb, s));
      RBT_HIP_CHECK(hipMemcpyAsync(hn.data(), nrm, nc * sizeof(double), hipMemcpyDeviceToHost, s));
      RBT_HIP_CHECK(hipStreamSynchronize(s));
      H.assign(size_t(nc) * (m + 1) * m, 0.0);
      cs.assign(size_t(nc) * m, 0.0);
      sn.assign(size_t(nc) * m, 0.0);
      gv.assign(size_t(nc) * (m + 1), 0.0);
      beta.assign(nc, 0.0);
      kc.assign(nc, 0);
      active.assign(nc, 0);
      hist.assign(size_t(nc) * (m + 1), 1.0);
      for (int c = 0; c < nc; ++c) {
        beta[c] = hn[c] > 0.0 ? std::sqrt(hn[c]) : 0.0;
        gv[size_t(c) * (m + 1)] = beta[c];
        active[c] = beta[c] > 0.0;
      }
      for (int j = 0; j < m && total < max_iter; ++j) {
        double *Vj = Vb + j * vs;
        {
          StageScope t(kStageResidual, s, 8.0 * double(n) * n);
          RBT_HIP_CHECK(launch_matvec(n, nc, A, lda, Vj, n, W, n, scratch, s));
        }
        rc = apply_solve(g, nc, LU, ldlu, W, n, U, V, winv, sync, true, s);
        if (rc) return rc;
        RBT_HIP_CHECK(launch_coldots(n, nc, j + 1, Vb, vs, W, n, dots, s));
        RBT_HIP_CHECK(launch_colcombo(n, nc, j + 1, Vb, vs, dots, -1.0, W, n, s));
        RBT_HIP_CHECK(launch_coldots(n, nc, j + 1, Vb, vs, W, n, dots2, s));
        RBT_HIP_CHECK(launch_colcombo(n, nc, j + 1, Vb, vs, dots2, -1.0, W, n, s));
        RBT_HIP_CHECK(launch_coldots(n, nc, 1, W, 0, W, n, nrm, s));
        RBT_HIP_CHECK(launch_colscale(n, nc, W, n, nrm, Vb + (j + 1) * vs, s));
        RBT_HIP_CHECK(hipMemcpyAsync(hd.data(), dots, (j + 1) * nc * sizeof(double),
                                     hipMemcpyDeviceToHost, s));
        RBT_HIP_CHECK(hipMemcpyAsync(hd2.data(), dots2, (j + 1) * nc * sizeof(double),
                                     hipMemcpyDeviceToHost, s));
        RBT_HIP_CHECK(hipMemcpyAsync(hn.data(), nrm, nc * sizeof(double), hipMemcpyDeviceToHost, s));
        RBT_HIP_CHECK(hipStreamSynchronize(s));
        ++total;
        bool all_done = true;
        for (int c = 0; c < nc; ++c) {
          if (!active[c]) continue;
          double *h = &H[(size_t(c) * m + j) * (m + 1)];  // column j of column c's Hessenberg
          for (int i = 0; i <= j; ++i) h[i] = hd[i * nc + c] + hd2[i * nc + c];
          h[j + 1] = hn[c] > 0.0 ? std::sqrt(hn[c]) : 0.0;
          double *csc = &cs[size_t(c) * m], *snc = &sn[size_t(c) * m];
          double *gc = &gv[size_t(c) * (m + 1)];
          for (int i = 0; i < j; ++i) {
            const double t0 = csc[i] * h[i] + snc[i] * h[i + 1];
            h[i + 1] = -snc[i] * h[i] + csc[i] * h[i + 1];
            h[i] = t0;
          }
          const double den = std::hypot(h[j], h[j + 1]);
          csc[j] = den > 0.0 ? h[j] / den : 1.0;
          snc[j] = den > 0.0 ? h[j + 1] / den : 0.0;
          const double sub = h[j + 1];
          h[j] = den;
          h[j + 1] = 0.0;
          gc[j + 1] = -snc[j] * gc[j];
          gc[j] = csc[j] * gc[j];
          kc[c] = j + 1;
          if (!(std::fabs(gc[j + 1]) > kGmresTau * beta[c]) || sub == 0.0 || den == 0.0)
            active[c] = 0;
          else
            all_done = false;
        }
        if (all_done) break;
        // guarded use: extrapolate each column's residual estimate at the
        // geometric rate of its last kGmresStallWin iterations over the
        // remaining budget; if that leaves the backward error far above tol,
        // stop (the caller falls back)
        if (stalled) {
          double pred = 0.0;
          for (int c = 0; c < nc; ++c) {
            const double r = beta[c] > 0.0 ? std::fabs(gv[size_t(c) * (m + 1) + j + 1]) / beta[c]
                                           : 0.0;
            hist[size_t(c) * (m + 1) + j + 1] = r;
            if (!active[c] || j + 1 < kGmresStallMin) continue;
            const double r0 = hist[size_t(c) * (m + 1) + j + 1 - kGmresStallWin];
            const double rate = r0 > 0.0 ? std::pow(r / r0, 1.0 / kGmresStallWin) : 0.0;
            const double p = r * std::pow(rate, double(max_iter - total));
            pred = p > pred ? p : pred;
          }
          if (be * pred > kGmresStallMargin * tol) {
            stop = true;
            break;
          }
        }
      }
      // y = R^-1 g per column (upper triangular, size kc[c]); X += V y
      int kmax = 0;
      y.assign(size_t(m + 1) * nc, 0.0);
      for (int c = 0; c < nc; ++c) {
        const int k = kc[c];
        kmax = k > kmax ? k : kmax;
        const double *gc = &gv[size_t(c) * (m + 1)];
        for (int i = k - 1; i >= 0; --i) {
          double acc = gc[i];
          for (int l = i + 1; l < k; ++l)
            acc -= H[(size_t(c) * m + l) * (m + 1) + i] * y[size_t(l) * nc + c];
          const double d = H[(size_t(c) * m + i) * (m + 1) + i];
          y[size_t(i) * nc + c] = d != 0.0 ? acc / d : 0.0;
        }
      }
      if (kmax > 0) {
        RBT_HIP_CHECK(hipMemcpyAsync(coef, y.data(), size_t(kmax) * nc * sizeof(double),
                                     hipMemcpyHostToDevice, s));
        RBT_HIP_CHECK(launch_colcombo(n, nc, kmax, Vb, vs, coef, 1.0, Xc, ldx, s));
        // y must stay valid until the copy has run: the residual that starts
        // the next step synchronizes the stream
      } else {
        break;  // no progress possible (zero preconditioned residual)
      }
      if (stop) {
        // the correction is kept; y is still read by the copy above
        RBT_HIP_CHECK(hipStreamSynchronize(s));
        *stalled = true;
        worst = total > worst ? total : worst;
        *it_out = worst;
        return residual(nrhs, X, B);
      }
    }
    worst = total > worst ? total : worst;
  }
  if (nrhs > kSkinnyMax) {  // backward error over all columns
    const int rc = residual(nrhs, X, B);
    if (rc) return rc;
  }
  *it_out = worst;
  return 0;
}

// ---- partial pivoting (the robust re-solve of the Sec. 5 fallback) ----

// R <- A^-1 R with the GEPP factors: R = P R (gathered through perm), then
// the triangular solves of the unpivoted factors (same L\U layout).
int gepp_apply(int64_t n, int64_t nrhs, const double *LU, int64_t ld, const int64_t *perm,
               double *R, int64_t ldr, double *ygat, const double *winv, int32_t *sync,
               hipStream_t s) {
  RBT_HIP_CHECK(launch_gather_rows(n, nrhs, perm, R, ldr, ygat, n, s));
  RBT_HIP_CHECK(launch_copy_cols(n, nrhs, ygat, n, R, ldr, s));
  return getrs_t(n, nrhs, LU, ld, R, ldr, 0, winv, sync, s);
}

// GEPP of A (copied into LU) and the solve X = A^-1 B, then classical FP64
// refinement with the GEPP factors until the Eq. 7 backward error is <= tol
// or max_iter corrections. ipiv, perm: n int64 each.
int gepp_solve_refine(int64_t n, int64_t nrhs, const double *A, int64_t lda, double *LU,
                      int64_t ldlu, const double *B, int64_t ldb, double *X, int64_t ldx,
                      double tol, int max_iter, int32_t *info, void *work, const Layout &L,
                      double *berr, int *it_out, hipStream_t s) {
  int64_t *ipiv = at<int64_t>(work, L.o_piv);
  int64_t *perm = ipiv + n;
  double *winv = at<double>(work, L.o_winv);
  int32_t *sync = at<int32_t>(work, L.o_sync);
  double *R = at<double>(work, L.o_resid);
  double *scratch = at<double>(work, L.o_partial);
  double *ygat = at<double>(work, L.o_ygat);
  double *anorm = at<double>(work, L.o_small);
  *it_out = 0;
  if (info) RBT_HIP_CHECK(launch_fill_i32(info, 0, s));
  RBT_HIP_CHECK(launch_copy_cols(n, n, A, lda, LU, ldlu, s));
  {
    StageScope t(kStagePivoted, s, 2.0 / 3.0 * double(n) * n * n);
    RBT_HIP_CHECK(launch_gepp(n, LU, ldlu, ipiv, info, at<char>(work, L.o_gscr), s));
  }
  RBT_HIP_CHECK(launch_ipiv_to_perm(n, ipiv, perm, s));
  int rc = diag_inverses_t(n, nrhs, LU, ldlu, winv, s);
  if (rc) return rc;
  RBT_HIP_CHECK(clear_sweep_err(sync, s));
  RBT_HIP_CHECK(launch_copy_cols(n, nrhs, B, ldb, X, ldx, s));
  rc = gepp_apply(n, nrhs, LU, ldlu, perm, X, ldx, ygat, winv, sync, s);
  if (rc) return rc;
  int it = 0;
  for (;;) {
    {
      StageScope t(kStageResidual, s, 8.0 * double(n) * n);
      RBT_HIP_CHECK(launch_residual_berr(n, nrhs, A, lda, X, ldx, B, ldb, R, n, it == 0, scratch,
                                         anorm, berr, s));
    }
    if (it >= max_iter) break;
    double be_host = 0.0;
    RBT_HIP_CHECK(hipMemcpyAsync(&be_host, berr, sizeof(double), hipMemcpyDeviceToHost, s));
    if (const int e = read_sweep_err(sync, s)) return e;
    if (be_host <= tol || !(be_host < HUGE_VAL)) break;
    rc = gepp_apply(n, nrhs, LU, ldlu, perm, R, n, ygat, winv, sync, s);
    if (rc) return rc;
    RBT_HIP_CHECK(launch_axpy_cols(n, nrhs, R, n, X, ldx, s));
    ++it;
  }
  *it_out = it;
  return read_sweep_err(sync, s);
}

bool bad_depth(int d) { return d < 0 || d > RBT_MAX_DEPTH; }

}  // namespace
}  // namespace rbt

using namespace rbt;

extern "C" size_t rbt_workspace_size(int64_t n, int64_t nrhs, int depth, int precision) {
  if (n < 0 || nrhs < 0 || bad_depth(depth)) return 0;
  if (precision != RBT_FP64 && precision != RBT_FP32 && precision != RBT_BF16) return 0;
  return layout(n, nrhs, depth, precision != RBT_FP64, precision == RBT_BF16).total_staged;
}

extern "C" int rbt_generate_device(int64_t n, int depth, uint64_t seed, double *dU, double *dV,
                                   void *stream) {
  if (n < 0) return -1;
  if (bad_depth(depth)) return -2;
  if (n > 0 && depth > 0 && dU == nullptr) return -4;
  if (n > 0 && depth > 0 && dV == nullptr) return -5;
  RBT_HIP_CHECK(launch_generate(geometry(n, depth), seed, dU, dV, S(stream)));
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
  if (n > 0 && depth > 0 && dU == nullptr) return -7;
  if (n > 0 && depth > 0 && dV == nullptr) return -8;
  if (bad_depth(depth)) return -9;
  RBT_HIP_CHECK(transform2_t(geometry(n, depth), A, lda, Out, ldo, out_prec, dU, dV, S(stream)));
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

extern "C" int rbt_genp(int64_t n, double *A, int64_t lda, int32_t *info_dev, void *stream) {
  if (n < 0) return -1;
  if (n > 0 && A == nullptr) return -2;
  if (lda < (n > 1 ? n : 1)) return -3;
  return genp_fp64(n, A, lda, info_dev, S(stream));
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
  const Layout L = layout(n, nrhs, 0);
  if (n > 0 && work == nullptr) return -8;
  if (work_bytes < L.o_sync + L.sync) return RBT_ERR_WORKSPACE;
  hipStream_t s = S(stream);
  double *winv = at<double>(work, L.o_winv);
  int32_t *sync = at<int32_t>(work, L.o_sync);
  RBT_HIP_CHECK(clear_sweep_err(sync, s));
  int rc = diag_inverses_t(n, nrhs, LU, ldlu, winv, s);
  if (rc) return rc;
  return getrs_fp64(n, nrhs, LU, ldlu, B, ldb, trans, winv, sync, s);
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
  RBT_HIP_CHECK(generate_t(n, depth, seed, U, V, s));
  RBT_HIP_CHECK(transform2_t(g, A, lda, A, lda, RBT_FP64, U, V, s));
  RBT_HIP_CHECK(transform_vec_t(g, nrhs, B, ldb, U, RBT_OP_T, s));
  double *winv = at<double>(work, L.o_winv);
  int rc = genp_fp64(n, A, lda, info_dev, s);
  if (rc) return rc;
  rc = diag_inverses_t(n, nrhs, A, lda, winv, s);
  if (rc) return rc;
  RBT_HIP_CHECK(clear_sweep_err(at<int32_t>(work, L.o_sync), s));
  rc = getrs_t(n, nrhs, A, lda, B, ldb, 0, winv, at<int32_t>(work, L.o_sync), s);
  if (rc) return rc;
  RBT_HIP_CHECK(transform_v_t(g, nrhs, B, ldb, V, RBT_OP_N, s));
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

// ---- allocation-free entry point ----
namespace rbt {
namespace {
// Workspace of rbt_solve_ex_noalloc: one array per GPU, held until the
// process ends. Host code never uses the array's name as an address: the
// device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kNoAllocBytes = size_t(RBT_NOALLOC_SCRATCH_MB) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Device address of `scratch` on the current device (looked up on the first
// call on each device, with that device current), or nullptr on failure.
void *scratch_ptr() {
  static std::mutex mu;
  static std::vector<void *> per_dev;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (per_dev.size() <= size_t(dev)) per_dev.resize(dev + 1, nullptr);
  if (per_dev[dev] == nullptr) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    per_dev[dev] = p;
  }
  return per_dev[dev];
}
}  // namespace
}  // namespace rbt

extern "C" int rbt_solve_ex_noalloc(int64_t n, int64_t nrhs, double *A, int64_t lda, double *B,
                                    int64_t ldb, int depth, uint64_t seed, int32_t *info_dev,
                                    void *stream) {
  if (n < 0) return -1;
  if (nrhs < 0) return -2;
  if (bad_depth(depth)) return -7;
  if (layout(n, nrhs, depth).total > kNoAllocBytes) return RBT_ERR_WORKSPACE;
  void *work = scratch_ptr();
  if (work == nullptr) return RBT_ERR_HIP;
  return rbt_solve_ex(n, nrhs, A, lda, B, ldb, depth, seed, info_dev, work, kNoAllocBytes, stream);
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
  double *scratch = at<double>(work, L.o_partial);
  double *small = at<double>(work, L.o_small);
  RBT_HIP_CHECK(launch_residual_berr(n, nrhs, A, lda, X, ldx, B, ldb, R, n, true, scratch, small,
                                     berr_dev, s));
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
  if (options().capturable && nrhs > kSkinnyMax) return RBT_ERR_UNSUPPORTED;
  const Layout L = layout(n, nrhs, depth);
  if (n > 0 && work == nullptr) return -18;
  if (work_bytes < L.total) return RBT_ERR_WORKSPACE;
  hipStream_t s = S(stream);
  double *small = at<double>(work, L.o_small);
  double *berr = berr_dev ? berr_dev : small + 1;
  if (n == 0 || nrhs == 0) {
    RBT_HIP_CHECK(launch_fill_f64(berr, 0.0, s));
    if (iters_dev) RBT_HIP_CHECK(launch_fill_i32(iters_dev, 0, s));
    return 0;
  }
  const Geometry g = geometry(n, depth);
  double *U = at<double>(work, L.o_coef);
  double *V = U + n * depth;
  double *R = at<double>(work, L.o_resid);
  double *scratch = at<double>(work, L.o_partial);
  double *anorm = small;

  RBT_HIP_CHECK(generate_t(n, depth, seed, U, V, s));
  RBT_HIP_CHECK(transform2_t(g, A, lda, LU, ldlu, RBT_FP64, U, V, s));
  double *winv = at<double>(work, L.o_winv);
  int rc = genp_fp64(n, LU, ldlu, info_dev, s);
  if (rc) return rc;
  rc = diag_inverses_t(n, nrhs, LU, ldlu, winv, s);
  if (rc) return rc;
  RBT_HIP_CHECK(launch_copy_cols(n, nrhs, B, ldb, X, ldx, s));
  int32_t *sync = at<int32_t>(work, L.o_sync);
  RBT_HIP_CHECK(clear_sweep_err(sync, s));
  rc = apply_solve(g, nrhs, (const double *)LU, ldlu, X, ldx, U, V, winv, sync, true, s);
  if (rc) return rc;
  if (options().capturable) {
    // no host test: an expired sweep wait shows as a NaN backward error
    int32_t *words = reinterpret_cast<int32_t *>(small + 32);
    return refine_classic_device(n, nrhs, A, lda, (const double *)LU, ldlu, B, ldb, X, ldx, g,
                                 U, V, winv, sync, R, scratch, anorm, berr, tol, max_iter,
                                 words, iters_dev ? iters_dev : words + 1, true, s);
  }
  int it = 0;
  rc = refine_classic(n, nrhs, A, lda, (const double *)LU, ldlu, B, ldb, X, ldx, g, U, V, winv, sync, R,
                      scratch, anorm, berr, tol, max_iter, &it, true, s);
  if (rc) return rc;
  if (iters_dev)
    RBT_HIP_CHECK(hipMemcpyAsync(iters_dev, &it, sizeof(int32_t), hipMemcpyHostToDevice, s));
  return read_sweep_err(sync, s);  // synchronizes
}

namespace rbt {
namespace {

// Body of the mixed-precision solve. stalled != nullptr: guarded use, the
// refinement stops early when it cannot reach tol (non-finite error, or no
// progress), *stalled says so. *it_out = refinement iterations.
int mixed_impl(int64_t n, int64_t nrhs, const double *A, int64_t lda, float *LU, int64_t ldlu,
               const double *B, int64_t ldb, double *X, int64_t ldx, int depth, uint64_t seed,
               int prec, int solver, double tol, int max_iter, double *berr_dev,
               int32_t *info_dev, void *work, size_t work_bytes, hipStream_t s, int *it_out,
               bool *stalled, int32_t *iters_cap = nullptr) {
  *it_out = 0;
  const Layout L = layout(n, nrhs, depth, true, prec == RBT_BF16);
  if (work_bytes < L.total) return RBT_ERR_WORKSPACE;
  // the BF16 operand staging area, when the caller's workspace holds it
  void *stage = (L.hstage > 0 && work_bytes >= L.total_staged) ? at<char>(work, L.o_hstage)
                                                                : nullptr;
  const size_t stage_bytes = stage ? L.hstage : 0;
  double *small = at<double>(work, L.o_small);
  double *berr = berr_dev ? berr_dev : small + 1;
  if (n == 0 || nrhs == 0) {
    RBT_HIP_CHECK(launch_fill_f64(berr, 0.0, s));
    if (iters_cap) RBT_HIP_CHECK(launch_fill_i32(iters_cap, 0, s));
    if (n > 0) {  // still factor, as the square case of rbt_genp
      const Geometry g = geometry(n, depth);
      double *U = at<double>(work, L.o_coef);
      RBT_HIP_CHECK(generate_t(n, depth, seed, U, U + n * depth, s));
      RBT_HIP_CHECK(transform2_t(g, A, lda, LU, ldlu, RBT_FP32, U, U + n * depth, s));
      return genp_impl(n, LU, ldlu, info_dev, prec, s, stage, stage_bytes);
    }
    if (info_dev) RBT_HIP_CHECK(launch_fill_i32(info_dev, 0, s));
    return 0;
  }
  const Geometry g = geometry(n, depth);
  double *U = at<double>(work, L.o_coef);
  double *V = U + n * depth;
  double *R = at<double>(work, L.o_resid);
  double *scratch = at<double>(work, L.o_partial);
  double *winv = at<double>(work, L.o_winv);
  double *anorm = small;

  RBT_HIP_CHECK(generate_t(n, depth, seed, U, V, s));
  RBT_HIP_CHECK(transform2_t(g, A, lda, LU, ldlu, RBT_FP32, U, V, s));
  int rc = genp_impl(n, LU, ldlu, info_dev, prec, s, stage, stage_bytes);
  if (rc) return rc;
  // triangular solves with the FP32 factors: FP32 arithmetic for classical
  // refinement; GMRES-IR applies its preconditioner in FP64 (also to the
  // first solve, so one set of inverses serves all of them)
  const bool f64 = options().mixed_fp64_inner != 0 || solver == RBT_IR_GMRES;
  rc = diag_inverses_t(n, LU, ldlu, winv, f64, s);
  if (rc) return rc;
  RBT_HIP_CHECK(launch_copy_cols(n, nrhs, B, ldb, X, ldx, s));
  int32_t *sync = at<int32_t>(work, L.o_sync);
  RBT_HIP_CHECK(clear_sweep_err(sync, s));
  rc = apply_solve(g, nrhs, (const float *)LU, ldlu, X, ldx, U, V, winv, sync, f64, s);
  if (rc) return rc;
  if (iters_cap != nullptr) {
    int32_t *words = reinterpret_cast<int32_t *>(small + 32);
    return refine_classic_device(n, nrhs, A, lda, (const float *)LU, ldlu, B, ldb, X, ldx, g, U,
                                 V, winv, sync, R, scratch, anorm, berr, tol, max_iter, words,
                                 iters_cap, f64, s);
  }
  if (solver == RBT_IR_GMRES)
    rc = refine_gmres(n, nrhs, A, lda, (const float *)LU, ldlu, B, ldb, X, ldx, g, U, V, winv,
                      sync, R, scratch, at<double>(work, L.o_krylov), anorm, berr, tol, max_iter,
                      it_out, s, stalled);
  else
    rc = refine_classic(n, nrhs, A, lda, (const float *)LU, ldlu, B, ldb, X, ldx, g, U, V, winv,
                        sync, R, scratch, anorm, berr, tol, max_iter, it_out, f64, s, stalled);
  if (rc) return rc;
  return read_sweep_err(sync, s);  // synchronizes
}

int mixed_args(int64_t n, int64_t nrhs, const double *A, int64_t lda, const float *LU,
               int64_t ldlu, const double *B, int64_t ldb, const double *X, int64_t ldx,
               int depth, int prec, int solver, double tol, int max_iter) {
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
  if (prec != RBT_FP32 && prec != RBT_BF16) return -13;
  if (solver != RBT_IR_CLASSIC && solver != RBT_IR_GMRES) return -14;
  if (!(tol >= 0.0)) return -15;
  if (max_iter < 0) return -16;
  return 0;
}

}  // namespace
}  // namespace rbt

extern "C" int rbt_solve_mixed(int64_t n, int64_t nrhs, const double *A, int64_t lda, float *LU,
                               int64_t ldlu, const double *B, int64_t ldb, double *X, int64_t ldx,
                               int depth, uint64_t seed, int prec, int solver, double tol,
                               int max_iter, int32_t *iters_dev, double *berr_dev,
                               int32_t *info_dev, void *work, size_t work_bytes, void *stream) {
  int rc = mixed_args(n, nrhs, A, lda, LU, ldlu, B, ldb, X, ldx, depth, prec, solver, tol,
                      max_iter);
  if (rc) return rc;
  if (n > 0 && work == nullptr) return -20;
  hipStream_t s = S(stream);
  int it = 0;
  if (options().capturable) {
    if (solver != RBT_IR_CLASSIC || nrhs > kSkinnyMax) return RBT_ERR_UNSUPPORTED;
    const Layout L = layout(n, nrhs, depth, true, prec == RBT_BF16);
    if (work_bytes < L.total) return RBT_ERR_WORKSPACE;
    int32_t *words = reinterpret_cast<int32_t *>(at<double>(work, L.o_small) + 32);
    return mixed_impl(n, nrhs, A, lda, LU, ldlu, B, ldb, X, ldx, depth, seed, prec, solver, tol,
                      max_iter, berr_dev, info_dev, work, work_bytes, s, &it, nullptr,
                      iters_dev ? iters_dev : words + 1);
  }
  rc = mixed_impl(n, nrhs, A, lda, LU, ldlu, B, ldb, X, ldx, depth, seed, prec, solver, tol,
                  max_iter, berr_dev, info_dev, work, work_bytes, s, &it, nullptr);
  if (rc) return rc;
  if (iters_dev) {
    RBT_HIP_CHECK(hipMemcpyAsync(iters_dev, &it, sizeof(int32_t), hipMemcpyHostToDevice, s));
    RBT_HIP_CHECK(hipStreamSynchronize(s));
  }
  return 0;
}

extern "C" int rbt_solve_mixed_guarded(int64_t n, int64_t nrhs, const double *A, int64_t lda,
                                       float *LU, int64_t ldlu, double *LU64, int64_t ldlu64,
                                       const double *B, int64_t ldb, double *X, int64_t ldx,
                                       int depth, uint64_t seed, int prec, int solver, double tol,
                                       int max_iter, int max_iter64, int32_t *iters_dev,
                                       double *berr_dev, int32_t *info_dev, int32_t *path_dev,
                                       void *work, size_t work_bytes, void *stream) {
  // argument numbers of rbt_solve_mixed shift by two after ldlu (LU64, ldlu64)
  int rc = mixed_args(n, nrhs, A, lda, LU, ldlu, B, ldb, X, ldx, depth, prec, solver, tol,
                      max_iter);
  if (rc <= -1 && rc >= -6) return rc;
  if (n > 0 && LU64 == nullptr) return -7;
  if (ldlu64 < (n > 1 ? n : 1)) return -8;
  if (rc <= -7 && rc >= -16) return rc - 2;
  if (rc) return rc;
  if (max_iter64 < 0) return -19;
  if (n > 0 && work == nullptr) return -24;
  hipStream_t s = S(stream);
  const Layout L = layout(n, nrhs, depth, true);
  if (work_bytes < L.total) return RBT_ERR_WORKSPACE;
  double *small = at<double>(work, L.o_small);
  double *berr = berr_dev ? berr_dev : small + 1;
  int32_t its[2] = {0, 0};
  int32_t path = 0;
  bool stalled = false;
  rc = mixed_impl(n, nrhs, A, lda, LU, ldlu, B, ldb, X, ldx, depth, seed, prec, solver, tol,
                  max_iter, berr, info_dev, work, work_bytes, s, &its[0], &stalled);
  if (rc) return rc;
  if (info_dev) RBT_HIP_CHECK(launch_fill_i32(info_dev + 1, 0, s));
  double be = 0.0;
  RBT_HIP_CHECK(hipMemcpyAsync(&be, berr, sizeof(double), hipMemcpyDeviceToHost, s));
  RBT_HIP_CHECK(hipStreamSynchronize(s));
  if (n > 0 && nrhs > 0 && !(be <= tol)) {
    // the low-precision factors cannot reach tol: factor A~ again in FP64
    // (same butterflies, already in the workspace) and refine from scratch
    path = 1;
    const Geometry g = geometry(n, depth);
    double *U = at<double>(work, L.o_coef);
    double *V = U + n * depth;
    double *winv = at<double>(work, L.o_winv);
    int32_t *sync = at<int32_t>(work, L.o_sync);
    RBT_HIP_CHECK(clear_sweep_err(sync, s));
    RBT_HIP_CHECK(transform2_t(g, A, lda, LU64, ldlu64, RBT_FP64, U, V, s));
    rc = genp_fp64(n, LU64, ldlu64, info_dev ? info_dev + 1 : nullptr, s);
    if (rc) return rc;
    rc = diag_inverses_t(n, nrhs, LU64, ldlu64, winv, s);
    if (rc) return rc;
    RBT_HIP_CHECK(launch_copy_cols(n, nrhs, B, ldb, X, ldx, s));
    rc = apply_solve(g, nrhs, (const double *)LU64, ldlu64, X, ldx, U, V, winv, sync, true, s);
    if (rc) return rc;
    int it64 = 0;
    bool stalled64 = false;
    rc = refine_classic(n, nrhs, A, lda, (const double *)LU64, ldlu64, B, ldb, X, ldx, g, U, V,
                        winv, sync, at<double>(work, L.o_resid), at<double>(work, L.o_partial),
                        small, berr, tol, max_iter64, &it64, true, s, &stalled64);
    if (rc) return rc;
    its[1] = it64;
    rc = read_sweep_err(sync, s);
    if (rc) return rc;
    RBT_HIP_CHECK(hipMemcpyAsync(&be, berr, sizeof(double), hipMemcpyDeviceToHost, s));
    RBT_HIP_CHECK(hipStreamSynchronize(s));
    if (!(be <= tol)) {
      // the transform itself fails on this matrix (Sec. 6.3): re-solve A
      // with partial pivoting into LU64 and refine with those factors
      path = 2;
      rc = gepp_solve_refine(n, nrhs, A, lda, LU64, ldlu64, B, ldb, X, ldx, tol, max_iter64,
                             info_dev ? info_dev + 1 : nullptr, work, L, berr, &it64, s);
      if (rc) return rc;
      its[1] = it64;
    }
  }
  if (iters_dev)
    RBT_HIP_CHECK(hipMemcpyAsync(iters_dev, its, sizeof(its), hipMemcpyHostToDevice, s));
  if (path_dev)
    RBT_HIP_CHECK(hipMemcpyAsync(path_dev, &path, sizeof(path), hipMemcpyHostToDevice, s));
  RBT_HIP_CHECK(hipStreamSynchronize(s));
  return 0;
}

extern "C" int rbt_gepp(int64_t n, double *A, int64_t lda, int64_t *ipiv_dev, int32_t *info_dev,
                        void *work, size_t work_bytes, void *stream) {
  if (n < 0) return -1;
  if (n > 0 && A == nullptr) return -2;
  if (lda < (n > 1 ? n : 1)) return -3;
  if (n > 0 && ipiv_dev == nullptr) return -4;
  if (n > 0 && work == nullptr) return -6;
  if (work_bytes < gepp_scratch_bytes()) return RBT_ERR_WORKSPACE;
  hipStream_t s = S(stream);
  if (info_dev) RBT_HIP_CHECK(launch_fill_i32(info_dev, 0, s));
  if (n == 0) return 0;
  StageScope t(kStagePivoted, s, 2.0 / 3.0 * double(n) * n * n);
  RBT_HIP_CHECK(launch_gepp(n, A, lda, ipiv_dev, info_dev, work, s));
  return 0;
}

extern "C" int rbt_gepp_solve(int64_t n, int64_t nrhs, const double *LU, int64_t ldlu,
                              const int64_t *ipiv_dev, double *B, int64_t ldb, void *work,
                              size_t work_bytes, void *stream) {
  if (n < 0) return -1;
  if (nrhs < 0) return -2;
  if (n > 0 && LU == nullptr) return -3;
  if (ldlu < (n > 1 ? n : 1)) return -4;
  if (n > 0 && ipiv_dev == nullptr) return -5;
  if (n > 0 && nrhs > 0 && B == nullptr) return -6;
  if (ldb < (n > 1 ? n : 1)) return -7;
  const Layout L = layout(n, nrhs, 0);
  if (n > 0 && work == nullptr) return -8;
  if (work_bytes < L.total) return RBT_ERR_WORKSPACE;
  if (n == 0 || nrhs == 0) return 0;
  hipStream_t s = S(stream);
  int64_t *perm = at<int64_t>(work, L.o_piv) + n;
  double *winv = at<double>(work, L.o_winv);
  int32_t *sync = at<int32_t>(work, L.o_sync);
  RBT_HIP_CHECK(clear_sweep_err(sync, s));
  RBT_HIP_CHECK(launch_ipiv_to_perm(n, ipiv_dev, perm, s));
  int rc = diag_inverses_t(n, nrhs, LU, ldlu, winv, s);
  if (rc) return rc;
  return gepp_apply(n, nrhs, LU, ldlu, perm, B, ldb, at<double>(work, L.o_ygat), winv, sync, s);
}

extern "C" int rbt_solve_guarded(int64_t n, int64_t nrhs, const double *A, int64_t lda,
                                 double *LU, int64_t ldlu, const double *B, int64_t ldb,
                                 double *X, int64_t ldx, int depth, uint64_t seed, double tol,
                                 int max_iter, int32_t *iters_dev, double *berr_dev,
                                 int32_t *info_dev, int32_t *path_dev, void *work,
                                 size_t work_bytes, void *stream) {
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
  if (n > 0 && work == nullptr) return -19;
  if (work_bytes < L.total) return RBT_ERR_WORKSPACE;
  hipStream_t s = S(stream);
  double *small = at<double>(work, L.o_small);
  double *berr = berr_dev ? berr_dev : small + 1;
  int32_t its[2] = {0, 0}, path = 0;
  if (info_dev) RBT_HIP_CHECK(launch_fill_i32(info_dev + 1, 0, s));
  if (n == 0 || nrhs == 0) {
    RBT_HIP_CHECK(launch_fill_f64(berr, 0.0, s));
    if (info_dev) RBT_HIP_CHECK(launch_fill_i32(info_dev, 0, s));
  } else {
    const Geometry g = geometry(n, depth);
    double *U = at<double>(work, L.o_coef);
    double *V = U + n * depth;
    double *winv = at<double>(work, L.o_winv);
    int32_t *sync = at<int32_t>(work, L.o_sync);
    RBT_HIP_CHECK(generate_t(n, depth, seed, U, V, s));
    RBT_HIP_CHECK(transform2_t(g, A, lda, LU, ldlu, RBT_FP64, U, V, s));
    int rc = genp_fp64(n, LU, ldlu, info_dev, s);
    if (rc) return rc;
    rc = diag_inverses_t(n, nrhs, LU, ldlu, winv, s);
    if (rc) return rc;
    RBT_HIP_CHECK(clear_sweep_err(sync, s));
    RBT_HIP_CHECK(launch_copy_cols(n, nrhs, B, ldb, X, ldx, s));
    rc = apply_solve(g, nrhs, (const double *)LU, ldlu, X, ldx, U, V, winv, sync, true, s);
    if (rc) return rc;
    int it = 0;
    bool stalled = false;
    rc = refine_classic(n, nrhs, A, lda, (const double *)LU, ldlu, B, ldb, X, ldx, g, U, V, winv,
                        sync, at<double>(work, L.o_resid), at<double>(work, L.o_partial), small,
                        berr, tol, max_iter, &it, true, s, &stalled);
    if (rc) return rc;
    its[0] = it;
    rc = read_sweep_err(sync, s);
    if (rc) return rc;
    double be = 0.0;
    RBT_HIP_CHECK(hipMemcpyAsync(&be, berr, sizeof(double), hipMemcpyDeviceToHost, s));
    RBT_HIP_CHECK(hipStreamSynchronize(s));
    if (!(be <= tol)) {
      path = 2;
      rc = gepp_solve_refine(n, nrhs, A, lda, LU, ldlu, B, ldb, X, ldx, tol, max_iter,
                             info_dev ? info_dev + 1 : nullptr, work, L, berr, &it, s);
      if (rc) return rc;
      its[1] = it;
    }
  }
  if (iters_dev)
    RBT_HIP_CHECK(hipMemcpyAsync(iters_dev, its, sizeof(its), hipMemcpyHostToDevice, s));
  if (path_dev)
    RBT_HIP_CHECK(hipMemcpyAsync(path_dev, &path, sizeof(path), hipMemcpyHostToDevice, s));
  RBT_HIP_CHECK(hipStreamSynchronize(s));
  return 0;
}

// ---- batched solves ----
namespace rbt {
namespace {

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    return 256;
  return cus;
}

}  // namespace
}  // namespace rbt

extern "C" size_t rbt_batched_workspace_size(int64_t batch, const int64_t *n,
                                             const int64_t *nrhs, int depth, int prec) {
  if (check_batch_sizes(batch, n, nrhs) != 0 || bad_depth(depth)) return 0;
  if (prec != RBT_FP32 && prec != RBT_BF16) return 0;
  return batch_plan_sizes(batch, n, nrhs, depth, nullptr).total;
}

extern "C" int rbt_batched_plan(int64_t batch, const int64_t *n, const int64_t *nrhs, int depth,
                                int prec, void *work, size_t work_bytes, void *stream) {
  const int rc = check_batch_sizes(batch, n, nrhs);
  if (rc) return rc;
  if (bad_depth(depth)) return -4;
  if (prec != RBT_FP32 && prec != RBT_BF16) return -5;
  if (work == nullptr) return -6;
  std::vector<BatchDesc> desc;
  const BatchPlanSizes z = batch_plan_sizes(batch, n, nrhs, depth, &desc);
  if (work_bytes < z.total) return RBT_ERR_WORKSPACE;
  const std::vector<char> host = batch_plan_image(batch, depth, prec, z, desc);
  hipStream_t s = S(stream);
  RBT_HIP_CHECK(hipMemcpyAsync(work, host.data(), host.size(), hipMemcpyHostToDevice, s));
  RBT_HIP_CHECK(hipStreamSynchronize(s));
  return 0;
}

extern "C" int rbt_solve_batched(int64_t batch, const double *const *A, const int64_t *lda,
                                 const double *const *B, const int64_t *ldb, double *const *X,
                                 const int64_t *ldx, int depth, uint64_t seed, int prec,
                                 double tol, int max_iter, int32_t *iters_dev, double *berr_dev,
                                 int32_t *info_dev, int32_t *path_dev, void *work,
                                 size_t work_bytes, void *stream) {
  if (batch < 0) return -1;
  if (batch > 0 && (A == nullptr || lda == nullptr)) return A == nullptr ? -2 : -3;
  if (batch > 0 && (B == nullptr || ldb == nullptr)) return B == nullptr ? -4 : -5;
  if (batch > 0 && (X == nullptr || ldx == nullptr)) return X == nullptr ? -6 : -7;
  if (bad_depth(depth)) return -8;
  if (prec != RBT_FP32 && prec != RBT_BF16) return -10;
  if (tol != tol) return -11;
  if (max_iter < 0) return -12;
  if (batch == 0) return 0;
  if (work == nullptr) return -17;
  if (work_bytes < kBatchTableOffset + size_t(batch) * sizeof(BatchDesc)) return RBT_ERR_WORKSPACE;
  const int64_t cap = options().batch_wgs_per_cu * int64_t(device_cus());
  const int grid = int(batch < cap ? batch : cap);
  RBT_HIP_CHECK(launch_batched(batch, work, work_bytes, A, lda, B, ldb, X, ldx, depth, seed, prec,
                               tol, max_iter, iters_dev, berr_dev, info_dev, path_dev, grid,
                               options().batch_ct2_min_n, S(stream)));
  return 0;
}

extern "C" int rbt_timing_enable(int on) {
  timing().on = (on != 0);
  return 0;
}

extern "C" int rbt_timing_read(int nstages, double *ms, int64_t *launches, double *work) {
  if (nstages < 0) return -1;
  TimingState &t = timing();
  std::lock_guard<std::mutex> lock(t.mu);
  double acc[kStageCount] = {};
  int rc = 0;
  for (auto &r : t.recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) rc = RBT_ERR_HIP;
    float e = 0.0f;
    if (rc == 0 && hipEventElapsedTime(&e, r.a, r.b) == hipSuccess) acc[r.stage] += e;
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  t.recs.clear();
  for (int i = 0; i < nstages && i < kStageCount; ++i) {
    if (ms) ms[i] = acc[i];
    if (launches) launches[i] = t.launches[i];
    if (work) work[i] = t.work[i];
  }
  for (int i = 0; i < kStageCount; ++i) {
    t.launches[i] = 0;
    t.work[i] = 0.0;
  }
  return rc;
}

extern "C" int rbt_solve_backward_mixed(int64_t n, int64_t nrhs, const float *LU, int64_t ldlu,
                                        const double *A, int64_t lda, const double *X,
                                        int64_t ldx, const double *G, int64_t ldg, double *dA,
                                        int64_t ldda, double *dB, int64_t lddb, int depth,
                                        uint64_t seed, double tol, int max_iter,
                                        int32_t *iters_dev, double *berr_dev, void *work,
                                        size_t work_bytes, void *stream) {
  if (n < 0) return -1;
  if (nrhs < 0) return -2;
  if (n > 0 && LU == nullptr) return -3;
  if (ldlu < (n > 1 ? n : 1)) return -4;
  if (n > 0 && nrhs > 0 && A == nullptr) return -5;
  if (lda < (n > 1 ? n : 1)) return -6;
  if (n > 0 && nrhs > 0 && dA != nullptr && X == nullptr) return -7;
  if (ldx < (n > 1 ? n : 1)) return -8;
  if (n > 0 && nrhs > 0 && G == nullptr) return -9;
  if (ldg < (n > 1 ? n : 1)) return -10;
  if (dA != nullptr && ldda < (n > 1 ? n : 1)) return -12;
  if (n > 0 && nrhs > 0 && dB == nullptr) return -13;
  if (lddb < (n > 1 ? n : 1)) return -14;
  if (bad_depth(depth)) return -15;
  if (!(tol >= 0.0)) return -17;
  if (max_iter < 0) return -18;
  const Layout L = layout(n, nrhs, depth, true);
  if (n > 0 && work == nullptr) return -21;
  if (work_bytes < L.total) return RBT_ERR_WORKSPACE;
  hipStream_t s = S(stream);
  double *small = at<double>(work, L.o_small);
  double *berr = berr_dev ? berr_dev : small + 1;
  if (n == 0 || nrhs == 0) {
    RBT_HIP_CHECK(launch_fill_f64(berr, 0.0, s));
    if (iters_dev) RBT_HIP_CHECK(launch_fill_i32(iters_dev, 0, s));
    return 0;
  }
  const Geometry g = geometry(n, depth);
  double *U = at<double>(work, L.o_coef);
  double *V = U + n * depth;
  double *winv = at<double>(work, L.o_winv);
  int32_t *sync = at<int32_t>(work, L.o_sync);
  double *R = at<double>(work, L.o_resid);
  double *scratch = at<double>(work, L.o_partial);
  double *anorm = small;
  // Lambda = A^-T G = U (A~^-T (V^T G)) with the FP32 factors of A~, then
  // refinement on A^T Lambda = G in FP64
  RBT_HIP_CHECK(generate_t(n, depth, seed, U, V, s));
  RBT_HIP_CHECK(clear_sweep_err(sync, s));
  const bool f64 = options().mixed_fp64_inner != 0;
  int rc = diag_inverses_t(n, LU, ldlu, winv, f64, s);
  if (rc) return rc;
  auto adjoint_solve = [&](double *Y, int64_t ldy) -> int {
    RBT_HIP_CHECK(transform_v_t(g, nrhs, Y, ldy, V, RBT_OP_T, s));
    const int r = getrs_t(n, nrhs, LU, ldlu, Y, ldy, 1, winv, sync, f64, s);
    if (r) return r;
    RBT_HIP_CHECK(transform_vec_t(g, nrhs, Y, ldy, U, RBT_OP_N, s));
    return 0;
  };
  RBT_HIP_CHECK(launch_copy_cols(n, nrhs, G, ldg, dB, lddb, s));
  rc = adjoint_solve(dB, lddb);
  if (rc) return rc;
  int it = 0;
  for (;;) {
    {
      StageScope t(kStageResidual, s, 8.0 * double(n) * n);
      RBT_HIP_CHECK(launch_residual_berr_T(n, nrhs, A, lda, dB, lddb, G, ldg, R, n, it == 0,
                                           scratch, anorm, berr, s));
    }
    if (it >= max_iter) break;
    double be_host = 0.0;
    RBT_HIP_CHECK(hipMemcpyAsync(&be_host, berr, sizeof(double), hipMemcpyDeviceToHost, s));
    if (const int e = read_sweep_err(sync, s)) return e;  // also waits for be_host
    if (be_host <= tol) break;
    rc = adjoint_solve(R, n);
    if (rc) return rc;
    RBT_HIP_CHECK(launch_axpy_cols(n, nrhs, R, n, dB, lddb, s));
    ++it;
  }
  if (dA != nullptr) {
    StageScope t(kStageOuter, s, 8.0 * double(n) * n);
    RBT_HIP_CHECK(launch_neg_outer(n, nrhs, dB, lddb, X, ldx, dA, ldda, s));
  }
  if (iters_dev)
    RBT_HIP_CHECK(hipMemcpyAsync(iters_dev, &it, sizeof(int32_t), hipMemcpyHostToDevice, s));
  return read_sweep_err(sync, s);  // synchronizes
}

extern "C" int rbt_set_option(int option, int64_t value) {
  switch (option) {
    case RBT_OPT_OUTER_NB:
      if (value < kNB || value % kNB != 0 || value > 16 * kNB) return -2;
      options().outer_nb = value;
      return 0;
    case RBT_OPT_BATCH_TILE_COLS:  // one tile count for every system
      if (value != 1 && value != 2) return -2;
      options().batch_ct2_min_n = value == 2 ? 0 : INT64_MAX;
      return 0;
    case RBT_OPT_BATCH_TILE_COLS2_MIN_N:
      if (value < 0) return -2;
      options().batch_ct2_min_n = value;
      return 0;
    case RBT_OPT_BATCH_WGS_PER_CU:
      if (value != 1 && value != 2) return -2;
      options().batch_wgs_per_cu = value;
      return 0;
    case RBT_OPT_LOOKAHEAD:
      if (value != 0 && value != 1) return -2;
      options().lookahead = value;
      return 0;
    case RBT_OPT_BF16_STAGED:
      if (value != 0 && value != 1) return -2;
      options().bf16_staged = value;
      return 0;
    case RBT_OPT_SWEEP_SPIN_LIMIT:
      options().sweep_spin_limit = value < 0 ? -1 : value;
      return 0;
    case RBT_OPT_MIXED_FP64_INNER:
      if (value != 0 && value != 1) return -2;
      options().mixed_fp64_inner = value;
      return 0;
    case RBT_OPT_GRANULE:
      if (value < 1 || value > (int64_t(1) << 30)) return -2;
      options().granule = value;
      return 0;
    case RBT_OPT_BUTTERFLY:
      if (value != 0 && value != 1) return -2;
      options().kind = value;
      return 0;
    case RBT_OPT_SIDES:
      if (value != 1 && value != 2) return -2;
      options().sides = value;
      return 0;
    case RBT_OPT_CAPTURABLE:
      if (value != 0 && value != 1) return -2;
      options().capturable = value;
      return 0;
    case RBT_OPT_PANEL_SPLIT:
      if (value < 0 || value > 2) return -2;
      options().panel_split = value;
      return 0;
    case RBT_OPT_TIMING_STAGES:
      if (value < 1 || value >= (int64_t(1) << kStageCount)) return -2;
      timing().mask = uint32_t(value);
      return 0;
    default:
      return -1;
  }
}

extern "C" int64_t rbt_get_option(int option) {
  switch (option) {
    case RBT_OPT_OUTER_NB: return options().outer_nb;
    case RBT_OPT_BATCH_TILE_COLS:
      return options().batch_ct2_min_n == 0 ? 2 : (options().batch_ct2_min_n == INT64_MAX ? 1 : 0);
    case RBT_OPT_BATCH_TILE_COLS2_MIN_N: return options().batch_ct2_min_n;
    case RBT_OPT_BATCH_WGS_PER_CU: return options().batch_wgs_per_cu;
    case RBT_OPT_LOOKAHEAD: return options().lookahead;
    case RBT_OPT_BF16_STAGED: return options().bf16_staged;
    case RBT_OPT_SWEEP_SPIN_LIMIT: return options().sweep_spin_limit;
    case RBT_OPT_MIXED_FP64_INNER: return options().mixed_fp64_inner;
    case RBT_OPT_GRANULE: return options().granule;
    case RBT_OPT_BUTTERFLY: return options().kind;
    case RBT_OPT_SIDES: return options().sides;
    case RBT_OPT_CAPTURABLE: return options().capturable;
    case RBT_OPT_PANEL_SPLIT: return options().panel_split;
    case RBT_OPT_TIMING_STAGES: return int64_t(timing().mask);
    default: return -1;
  }
}

extern "C" int rbt_solve_backward(int64_t n, int64_t nrhs, const double *LU, int64_t ldlu,
                                  const double *X, int64_t ldx, const double *G, int64_t ldg,
                                  double *dA, int64_t ldda, double *dB, int64_t lddb, int depth,
                                  uint64_t seed, void *work, size_t work_bytes, void *stream) {
  if (n < 0) return -1;
  if (nrhs < 0) return -2;
  if (n > 0 && LU == nullptr) return -3;
  if (ldlu < (n > 1 ? n : 1)) return -4;
  if (n > 0 && nrhs > 0 && dA != nullptr && X == nullptr) return -5;
  if (ldx < (n > 1 ? n : 1)) return -6;
  if (n > 0 && nrhs > 0 && G == nullptr) return -7;
  if (ldg < (n > 1 ? n : 1)) return -8;
  if (dA != nullptr && ldda < (n > 1 ? n : 1)) return -10;
  if (n > 0 && nrhs > 0 && dB == nullptr) return -11;
  if (lddb < (n > 1 ? n : 1)) return -12;
  if (bad_depth(depth)) return -13;
  const Layout L = layout(n, nrhs, depth);
  if (n > 0 && work == nullptr) return -15;
  if (work_bytes < L.total) return RBT_ERR_WORKSPACE;
  if (n == 0) return 0;
  hipStream_t s = S(stream);
  const Geometry g = geometry(n, depth);
  double *U = at<double>(work, L.o_coef);
  double *V = U + n * depth;
  double *winv = at<double>(work, L.o_winv);
  // Lambda = A^-T G = U (A~^-T (V^T G)),  A~ = U^T A V = L U_f
  RBT_HIP_CHECK(generate_t(n, depth, seed, U, V, s));
  RBT_HIP_CHECK(launch_copy_cols(n, nrhs, G, ldg, dB, lddb, s));
  RBT_HIP_CHECK(transform_v_t(g, nrhs, dB, lddb, V, RBT_OP_T, s));
  int rc = diag_inverses_t(n, nrhs, LU, ldlu, winv, s);
  if (rc) return rc;
  RBT_HIP_CHECK(clear_sweep_err(at<int32_t>(work, L.o_sync), s));
  rc = getrs_t(n, nrhs, LU, ldlu, dB, lddb, 1, winv, at<int32_t>(work, L.o_sync), s);
  if (rc) return rc;
  RBT_HIP_CHECK(transform_vec_t(g, nrhs, dB, lddb, U, RBT_OP_N, s));
  if (dA != nullptr) {
    StageScope t(kStageOuter, s, 8.0 * double(n) * n);
    RBT_HIP_CHECK(launch_neg_outer(n, nrhs, dB, lddb, X, ldx, dA, ldda, s));
  }
  return 0;
}
