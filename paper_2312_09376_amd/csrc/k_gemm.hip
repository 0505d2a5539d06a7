// FP64 matrix-core GEMM for gfx950: C (M x N) = A B or C -= A B, column-major.
//
// Used for the trailing update of the blocked elimination (A22 -= L21 U12,
// K = block size) and, with a triangular operand taken from a packed block
// inverse, for the block triangular solves (L21 = A21 U11^-1,
// U12 = L11^-1 A12, and the forward/backward solves).
//
// Tiling: 256 threads = 4 wavefronts in a 2 x 2 grid, block tile 128 x 128,
// wavefront tile 64 x 64 = 4 x 4 MFMA tiles of v_mfma_f64_16x16x4_f64,
// K staged through LDS in slices of 16 with a register-prefetched double
// buffer (one barrier per slice). The depth-128 updates inside and beside
// the panel use 64 x 64 block tiles instead (k_dgemm_small).
//
// Operand order: each MFMA computes a 16 x 16 tile of C^T (first operand a
// B^T fragment, second an A^T fragment). The accumulator layout of the f64
// instruction (lane l, element v holds output row l/16 + 4v, column l % 16;
// checked on the device) then gives every group of 16 lanes 16 consecutive
// rows of one column of C, so epilogue loads and stores are 128-byte
// contiguous runs.
//
// In place: when C aliases A (or B) the caller guarantees that a block tile
// reads only the rows (columns) it writes, i.e. N <= 128 (M <= 128); all
// reads of the K loop complete before the epilogue writes.
//
// Block ids are remapped so that each XCD (gfx950 dispatches workgroups
// round-robin over its 8 XCDs) receives a contiguous range of tiles, and
// that range is walked in groups of 8 tile rows: the ~64 workgroups resident
// on one XCD then cover an 8 x 8 block of C tiles and share 8 row panels of
// A and 8 column panels of B through the XCD's L2, instead of streaming a
// different A panel per workgroup.
#include "internal.h"

namespace rbt {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int GM = 8;    // tile rows per ordering group
constexpr int PADA = 4;  // As row stride BM + 4 doubles
constexpr int PADB = 1;  // Bs row stride BK + 1 doubles (odd: conflict-free column reads)

// Effective A(m, k) for the operand modes.
template <OpA OA>
__device__ __forceinline__ double load_a(const double *A, int64_t lda, int64_t m, int64_t k,
                                         int64_t M, int64_t K) {
  if (m >= M || k >= K) return 0.0;
  if constexpr (OA == OpA::General) {
    return A[m + k * lda];
  } else if constexpr (OA == OpA::GeneralT) {
    return A[k + m * lda];
  } else if constexpr (OA == OpA::UnitLower) {
    return m > k ? A[m + k * lda] : (m == k ? 1.0 : 0.0);
  } else if constexpr (OA == OpA::Upper) {
    return m <= k ? A[m + k * lda] : 0.0;
  } else if constexpr (OA == OpA::UnitLowerT) {
    return k > m ? A[k + m * lda] : (m == k ? 1.0 : 0.0);
  } else {  // UpperT
    return k <= m ? A[k + m * lda] : 0.0;
  }
}

template <OpB OB>
__device__ __forceinline__ double load_b(const double *B, int64_t ldb, int64_t k, int64_t n,
                                         int64_t K, int64_t N) {
  if (k >= K || n >= N) return 0.0;
  if constexpr (OB == OpB::General) {
    return B[k + n * ldb];
  } else {  // Upper
    return k <= n ? B[k + n * ldb] : 0.0;
  }
}

// A storage is contiguous along m for General/UnitLower/Upper, along k for
// the transposed modes; pick the load pattern that coalesces.
template <OpA OA>
constexpr bool a_m_contiguous() {
  return OA == OpA::General || OA == OpA::UnitLower || OA == OpA::Upper;
}

// One 128 x 128 block tile at (m0, n0). FAST: an interior tile of the plain
// product with K a multiple of BK (the kernel checks), which takes the
// unguarded loads in every slice and the whole-tile epilogue with no
// per-slice branches between the matrix-core blocks (3 % faster than
// choosing the load path slice by slice); every other tile takes the
// general body. Both compute the same products in the same order.
template <OpA OA, OpB OB, Acc AC, bool FAST>
__device__ __forceinline__ void dgemm_tile(int64_t M, int64_t N, int64_t K, const double *A,
                                           int64_t lda, const double *B, int64_t ldb, double *C,
                                           int64_t ldc, int64_t m0, int64_t n0,
                                           double (&As)[2][BK][BM + PADA],
                                           double (&Bs)[2][BN][BK + PADB]) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int l16 = lane & 15, lk = lane >> 4;

  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  // per-thread load coordinates
  // A, m-contiguous: 4 passes, each: column (tid / 64) + 4p, rows 2 (tid % 64) + {0,1}
  // A, k-contiguous: row m = tid / 2, k = 8 (tid % 2) + 0..7
  // B: column n = tid / 2, k = 8 (tid % 2) + 0..7
  double ra[8], rb[8];

  // Interior tiles of the plain product take unguarded 16-byte loads (the
  // operands are only 8-byte aligned in general, which these loads accept);
  // edge tiles and the last, partial K slice take the guarded path.
  const bool interior = FAST || ((OA == OpA::General) && (OB == OpB::General) &&
                                  (m0 + BM <= M) && (n0 + BN <= N));
  auto load_stage_fast = [&](int64_t k0) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int64_t k = k0 + (tid >> 6) + 4 * p;
      const d2u v = *reinterpret_cast<const d2u *>(A + (m0 + 2 * (tid & 63)) + k * lda);
      ra[2 * p] = v[0];
      ra[2 * p + 1] = v[1];
    }
    const double *bp = B + (k0 + 8 * (tid & 1)) + (n0 + (tid >> 1)) * ldb;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const d2u v = *reinterpret_cast<const d2u *>(bp + 2 * p);
      rb[2 * p] = v[0];
      rb[2 * p + 1] = v[1];
    }
  };

  // Edge tiles of the plain product: rows >= M and columns >= N only feed
  // outputs that are never stored, so they are read at clamped addresses
  // inside A and B with the same 16-byte loads (a row pair at r reads rows
  // rc, rc + 1 with rc = min(r, M - 2): row r's value is the first or the
  // second of them).
  const bool clamped = (OA == OpA::General) && (OB == OpB::General) && !interior && M >= 2;
  auto load_stage_clamped = [&](int64_t k0) {
    const int64_t r = m0 + 2 * (tid & 63);
    const int64_t rc = r < M - 1 ? r : M - 2;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int64_t k = k0 + (tid >> 6) + 4 * p;
      const d2u v = *reinterpret_cast<const d2u *>(A + rc + k * lda);
      ra[2 * p] = r == rc ? v[0] : v[1];
      ra[2 * p + 1] = v[1];
    }
    const int64_t nb = n0 + (tid >> 1);
    const double *bp = B + (k0 + 8 * (tid & 1)) + (nb < N ? nb : N - 1) * ldb;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const d2u v = *reinterpret_cast<const d2u *>(bp + 2 * p);
      rb[2 * p] = v[0];
      rb[2 * p + 1] = v[1];
    }
  };

  auto load_stage = [&](int64_t k0) {
    if constexpr (FAST) {
      load_stage_fast(k0);
      return;
    }
    if (k0 + BK <= K) {
      if (interior) {
        load_stage_fast(k0);
        return;
      }
      if (clamped) {
        load_stage_clamped(k0);
        return;
      }
    }
    if constexpr (a_m_contiguous<OA>()) {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int64_t k = k0 + (tid >> 6) + 4 * p;
        const int64_t m = m0 + 2 * (tid & 63);
        ra[2 * p] = load_a<OA>(A, lda, m, k, M, K);
        ra[2 * p + 1] = load_a<OA>(A, lda, m + 1, k, M, K);
      }
    } else {
      const int64_t m = m0 + (tid >> 1);
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const int64_t k = k0 + 8 * (tid & 1) + p;
        ra[p] = load_a<OA>(A, lda, m, k, M, K);
      }
    }
    const int64_t n = n0 + (tid >> 1);
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int64_t k = k0 + 8 * (tid & 1) + p;
      rb[p] = load_b<OB>(B, ldb, k, n, K, N);
    }
  };

  auto store_stage = [&](int s) {
    if constexpr (a_m_contiguous<OA>()) {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int k = (tid >> 6) + 4 * p;
        const int m = 2 * (tid & 63);
        As[s][k][m] = ra[2 * p];
        As[s][k][m + 1] = ra[2 * p + 1];
      }
    } else {
      const int m = tid >> 1;
#pragma unroll
      for (int p = 0; p < 8; ++p) As[s][8 * (tid & 1) + p][m] = ra[p];
    }
    const int n = tid >> 1;
#pragma unroll
    for (int p = 0; p < 8; ++p) Bs[s][n][8 * (tid & 1) + p] = rb[p];
  };

  load_stage(0);
  store_stage(0);
  __syncthreads();

  int cur = 0;
  for (int64_t k0 = 0; k0 < K; k0 += BK) {
    const bool has_next = k0 + BK < K;
    if (has_next) load_stage(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      double af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = As[cur][kk * 4 + lk][wm * 64 + i * 16 + l16];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = Bs[cur][wn * 64 + j * 16 + l16][kk * 4 + lk];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[j], af[i], acc[i][j], 0, 0, 0);
    }
    if (has_next) store_stage(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }

  // epilogue: lane holds C[m0 + wm*64 + i*16 + l16][n0 + wn*64 + j*16 + lk + 4*v].
  // The C values of row block i + 1 are loaded before row block i is
  // stored, so 16 loads per lane are in flight at a time (a load of C cannot
  // be moved above a store to C by the compiler, which would otherwise cost
  // one round trip per element). Edge tiles load at clamped addresses inside
  // C and store only their elements inside it.
  const int64_t r0 = m0 + wm * 64 + l16, c0 = n0 + wn * 64 + lk;
  if (FAST || (m0 + BM <= M && n0 + BN <= N)) {
    double *cp = C + r0 + c0 * ldc;
    if constexpr (AC == Acc::Overwrite) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) cp[i * 16 + (j * 16 + 4 * v) * ldc] = acc[i][j][v];
    } else {
      double cv[2][16];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) cv[0][4 * j + v] = cp[(j * 16 + 4 * v) * ldc];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (i + 1 < 4) {
#pragma unroll
          for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              cv[(i + 1) & 1][4 * j + v] = cp[(i + 1) * 16 + (j * 16 + 4 * v) * ldc];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            cp[i * 16 + (j * 16 + 4 * v) * ldc] = cv[i & 1][4 * j + v] - acc[i][j][v];
      }
    }
    return;
  }
  // edge tile: one column offset per (j, v) (clamped), rows per i
  int64_t coff[16];
  bool cin[16];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t col = c0 + j * 16 + 4 * v;
      cin[4 * j + v] = col < N;
      coff[4 * j + v] = (col < N ? col : N - 1) * ldc;
    }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = r0 + i * 16;
    if (row >= M) continue;
    double *cr = C + row;
    if constexpr (AC == Acc::Overwrite) {
#pragma unroll
      for (int e = 0; e < 16; ++e)
        if (cin[e]) cr[coff[e]] = acc[i][e >> 2][e & 3];
    } else {
      double cv[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) cv[e] = cr[coff[e]];
#pragma unroll
      for (int e = 0; e < 16; ++e)
        if (cin[e]) cr[coff[e]] = cv[e] - acc[i][e >> 2][e & 3];
    }
  }
}

// WHOLE: every tile is interior and K a multiple of BK (the launcher
// checks), so the kernel holds only the fast tile body (its registers are
// then allocated for that body alone: 1 % faster on the trailing updates).
template <OpA OA, OpB OB, Acc AC, bool WHOLE = false>
__global__ void __launch_bounds__(256, 2)
    k_dgemm(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda, const double *B,
            int64_t ldb, double *C, int64_t ldc, int tiles_m,
            int total) {
  __shared__ double As[2][BK][BM + PADA];
  __shared__ double Bs[2][BN][BK + PADB];

  // XCD-aware remap, then grouped tile order (groups of GM tile rows,
  // column-major inside a group)
  int pid = blockIdx.x;
  const int full = (total / 8) * 8;
  if (pid < full) pid = (pid % 8) * (total / 8) + pid / 8;
  const int tiles_n = total / tiles_m;
  const int group = pid / (GM * tiles_n);
  const int first_m = group * GM;
  const int gsize = (tiles_m - first_m) < GM ? (tiles_m - first_m) : GM;
  const int in_group = pid - group * GM * tiles_n;
  const int tm = first_m + in_group % gsize, tn = in_group / gsize;
  const int64_t m0 = int64_t(tm) * BM, n0 = int64_t(tn) * BN;

  if constexpr (OA == OpA::General && OB == OpB::General) {
    if (WHOLE || (m0 + BM <= M && n0 + BN <= N && K % BK == 0)) {
      dgemm_tile<OA, OB, AC, true>(M, N, K, A, lda, B, ldb, C, ldc, m0, n0, As, Bs);
      return;
    }
  }
  if constexpr (!WHOLE)
    dgemm_tile<OA, OB, AC, false>(M, N, K, A, lda, B, ldb, C, ldc, m0, n0, As, Bs);
}

// Small tiles for the updates inside and beside the panel (C -= A B with
// K = 128 and one dimension of at most 896): 64 x 64 block tiles, 4
// wavefronts of 32 x 32 (2 x 2 MFMA tiles), K in slices of 16, 34 KB of LDS
// so that four workgroups share a CU. A grid of 128 x 128 tiles leaves most
// CUs idle or with one tile for these shapes; four times as many tiles of a
// quarter of the work fill the chip and overlap one tile's prologue and
// epilogue with the others' matrix-core work. Every output element
// accumulates the same products in the same order as with the large tiles,
// so the result is identical.
constexpr int SM = 64, SN = 64, SK = 16;

// One 64 x 64 block tile at (m0, n0); FAST as for the large tiles (an
// interior tile with K a multiple of SK: plain loads, whole-tile epilogue,
// no per-slice branches; 8-10 % faster on the panel shapes).
template <Acc AC, bool FAST>
__device__ __forceinline__ void small_tile(int64_t M, int64_t N, int64_t K, const double *A,
                                           int64_t lda, const double *B, int64_t ldb, double *C,
                                           int64_t ldc, int64_t m0, int64_t n0,
                                           double (&As)[2][SK][SM + PADA],
                                           double (&Bs)[2][SN][SK + PADB]) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int l16 = lane & 15, lk = lane >> 4;

  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  // A slice (64 x 16): rows 2 (tid % 32) + {0,1}, columns tid / 32 + {0, 8};
  // B slice (16 x 64): column tid / 4, rows 4 (tid % 4) + 0..3
  double ra[4], rb[4];
  const bool interior = FAST || ((m0 + SM <= M) && (n0 + SN <= N));
  auto load_stage = [&](int64_t k0) {
    const int64_t ma = m0 + 2 * (tid & 31), ka = k0 + (tid >> 5);
    const int64_t nb = n0 + (tid >> 2), kb = k0 + 4 * (tid & 3);
    if constexpr (FAST) {
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const d2u v = *reinterpret_cast<const d2u *>(A + ma + (ka + 8 * p) * lda);
        ra[2 * p] = v[0];
        ra[2 * p + 1] = v[1];
      }
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const d2u v = *reinterpret_cast<const d2u *>(B + (kb + 2 * p) + nb * ldb);
        rb[2 * p] = v[0];
        rb[2 * p + 1] = v[1];
      }
      return;
    }
    if (k0 + SK <= K && (interior || M >= 2)) {
      // edge tiles read rows >= M and columns >= N (outputs never stored) at
      // clamped addresses: a row pair at ma reads rows mc, mc + 1, mc =
      // min(ma, M - 2), and row ma's value is the first or second of them
      const int64_t mc = ma < M - 1 ? ma : M - 2;
      const int64_t nc = nb < N ? nb : N - 1;
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const d2u v = *reinterpret_cast<const d2u *>(A + mc + (ka + 8 * p) * lda);
        ra[2 * p] = ma == mc ? v[0] : v[1];
        ra[2 * p + 1] = v[1];
      }
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const d2u v = *reinterpret_cast<const d2u *>(B + (kb + 2 * p) + nc * ldb);
        rb[2 * p] = v[0];
        rb[2 * p + 1] = v[1];
      }
      return;
    }
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      ra[2 * p] = load_a<OpA::General>(A, lda, ma, ka + 8 * p, M, K);
      ra[2 * p + 1] = load_a<OpA::General>(A, lda, ma + 1, ka + 8 * p, M, K);
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) rb[p] = load_b<OpB::General>(B, ldb, kb + p, nb, K, N);
  };
  auto store_stage = [&](int s) {
    const int ma = 2 * (tid & 31), ka = tid >> 5;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      As[s][ka + 8 * p][ma] = ra[2 * p];
      As[s][ka + 8 * p][ma + 1] = ra[2 * p + 1];
    }
    const int nb = tid >> 2, kb = 4 * (tid & 3);
#pragma unroll
    for (int p = 0; p < 4; ++p) Bs[s][nb][kb + p] = rb[p];
  };

  load_stage(0);
  store_stage(0);
  __syncthreads();
  int cur = 0;
  for (int64_t k0 = 0; k0 < K; k0 += SK) {
    const bool has_next = k0 + SK < K;
    if (has_next) load_stage(k0 + SK);
#pragma unroll
    for (int kk = 0; kk < SK / 4; ++kk) {
      double af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) af[i] = As[cur][kk * 4 + lk][wm * 32 + i * 16 + l16];
#pragma unroll
      for (int j = 0; j < 2; ++j) bf[j] = Bs[cur][wn * 32 + j * 16 + l16][kk * 4 + lk];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[j], af[i], acc[i][j], 0, 0, 0);
    }
    if (has_next) store_stage(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }

  // epilogue: lane holds C[m0 + wm*32 + i*16 + l16][n0 + wn*32 + j*16 + lk + 4*v]
  const int64_t r0 = m0 + wm * 32 + l16, c0 = n0 + wn * 32 + lk;
  if (interior) {
    double *cp = C + r0 + c0 * ldc;
    double cv[2][2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) cv[i][j][v] = cp[i * 16 + (j * 16 + 4 * v) * ldc];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) cp[i * 16 + (j * 16 + 4 * v) * ldc] = cv[i][j][v] - acc[i][j][v];
    return;
  }
  // edge tile: loads at clamped columns, stores inside C only
  int64_t coff[8];
  bool cin[8];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t col = c0 + j * 16 + 4 * v;
      cin[4 * j + v] = col < N;
      coff[4 * j + v] = (col < N ? col : N - 1) * ldc;
    }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int64_t row = r0 + i * 16;
    if (row >= M) continue;
    double *cr = C + row;
    double cv[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) cv[e] = cr[coff[e]];
#pragma unroll
    for (int e = 0; e < 8; ++e)
      if (cin[e]) cr[coff[e]] = cv[e] - acc[i][e >> 2][e & 3];
  }
}

// Tile `bid` of a grid of `total` 64 x 64 tiles over C (M x N), with the
// same XCD-aware and grouped order as the large tiles.
template <Acc AC>
__device__ __forceinline__ void small_grid_tile(int bid, int64_t M, int64_t N, int64_t K,
                                                const double *A, int64_t lda, const double *B,
                                                int64_t ldb, double *C, int64_t ldc, int tiles_m,
                                                int total, double (&As)[2][SK][SM + PADA],
                                                double (&Bs)[2][SN][SK + PADB]) {
  int pid = bid;
  const int full = (total / 8) * 8;
  if (pid < full) pid = (pid % 8) * (total / 8) + pid / 8;
  const int tiles_n = total / tiles_m;
  const int group = pid / (GM * tiles_n);
  const int first_m = group * GM;
  const int gsize = (tiles_m - first_m) < GM ? (tiles_m - first_m) : GM;
  const int in_group = pid - group * GM * tiles_n;
  const int tm = first_m + in_group % gsize, tn = in_group / gsize;
  const int64_t m0 = int64_t(tm) * SM, n0 = int64_t(tn) * SN;

  if (m0 + SM <= M && n0 + SN <= N && K % SK == 0)
    small_tile<AC, true>(M, N, K, A, lda, B, ldb, C, ldc, m0, n0, As, Bs);
  else
    small_tile<AC, false>(M, N, K, A, lda, B, ldb, C, ldc, m0, n0, As, Bs);
}

template <Acc AC>
__global__ void __launch_bounds__(256, 4)
    k_dgemm_small(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda,
                  const double *B, int64_t ldb, double *C, int64_t ldc, int tiles_m, int total) {
  __shared__ double As[2][SK][SM + PADA];
  __shared__ double Bs[2][SN][SK + PADB];
  small_grid_tile<AC>(int(blockIdx.x), M, N, K, A, lda, B, ldb, C, ldc, tiles_m, total, As, Bs);
}

// Two updates C -= A B of one depth K and one leading dimension in one
// launch: workgroups [0, start1) take the tiles of the first (the ids
// beyond its tile count exit; start1 is a multiple of 8 so that both keep
// their XCD order), the rest those of the second. Each tile computes what
// it computes in a launch of its own.
struct SubGemm {
  int64_t M, N;
  const double *A, *B;
  double *C;
  int tiles_m, total;
};

__global__ void __launch_bounds__(256, 4)
    k_dgemm_small2(int64_t K, int64_t ld, SubGemm p0, SubGemm p1, int start1) {
  __shared__ double As[2][SK][SM + PADA];
  __shared__ double Bs[2][SN][SK + PADB];
  int bid = int(blockIdx.x);
  if (bid >= start1) {
    bid -= start1;
    small_grid_tile<Acc::Subtract>(bid, p1.M, p1.N, K, p1.A, ld, p1.B, ld, p1.C, ld, p1.tiles_m,
                                   p1.total, As, Bs);
  } else if (bid < p0.total) {
    small_grid_tile<Acc::Subtract>(bid, p0.M, p0.N, K, p0.A, ld, p0.B, ld, p0.C, ld, p0.tiles_m,
                                   p0.total, As, Bs);
  }
}

hipError_t launch_small(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda,
                        const double *B, int64_t ldb, double *C, int64_t ldc, hipStream_t s) {
  const int64_t tm = (M + SM - 1) / SM, tn = (N + SN - 1) / SN;
  const int64_t total = tm * tn;
  if (total > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_dgemm_small<Acc::Subtract>), dim3(unsigned(total)), dim3(256), 0, s, M, N,
                     K, A, lda, B, ldb, C, ldc, int(tm), int(total));
  return hipGetLastError();
}

SubGemm sub_gemm(int64_t M, int64_t N, const double *A, const double *B, double *C) {
  SubGemm g{M, N, A, B, C, 0, 0};
  if (M > 0 && N > 0) {
    g.tiles_m = int((M + SM - 1) / SM);
    g.total = int(int64_t(g.tiles_m) * ((N + SN - 1) / SN));
  }
  return g;
}

template <OpA OA, OpB OB, Acc AC>
hipError_t launch_t(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda,
                    const double *B, int64_t ldb, double *C, int64_t ldc, hipStream_t s) {
  const int64_t tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN;
  const int64_t total = tm * tn;
  if (total > 0x7fffffff) return hipErrorInvalidValue;
  if constexpr (OA == OpA::General && OB == OpB::General && AC == Acc::SubtractTrailing) {
    if (M % BM == 0 && N % BN == 0 && K % BK == 0) {
      hipLaunchKernelGGL((k_dgemm<OA, OB, AC, true>), dim3(unsigned(total)), dim3(256), 0, s, M, N,
                         K, A, lda, B, ldb, C, ldc, int(tm), int(total));
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_dgemm<OA, OB, AC>), dim3(unsigned(total)), dim3(256), 0, s, M, N, K, A,
                     lda, B, ldb, C, ldc, int(tm), int(total));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_dgemm_tiles(int tile, int64_t M, int64_t N, int64_t K, const double *A,
                              int64_t lda, const double *B, int64_t ldb, double *C, int64_t ldc,
                              hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  if (tile == 64) return launch_small(M, N, K, A, lda, B, ldb, C, ldc, s);
  return launch_t<OpA::General, OpB::General, Acc::SubtractTrailing>(M, N, K, A, lda, B, ldb, C,
                                                                     ldc, s);
}

hipError_t launch_dgemm(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda, OpA opa,
                        const double *B, int64_t ldb, OpB opb, double *C, int64_t ldc, Acc acc,
                        hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (K <= 0) {
    if (acc != Acc::Overwrite) return hipSuccess;
    return hipErrorInvalidValue;  // C = 0 is never requested by the solver
  }
  // the updates inside and beside the panel (and of the block solves) run
  // on the small tiles, the trailing update on the large ones
  if (opa == OpA::General && opb == OpB::General && acc == Acc::Subtract)
    return launch_small(M, N, K, A, lda, B, ldb, C, ldc, s);
#define RBT_GEMM_CASE(OA_, OB_, AC_)                                              \
  if (opa == OA_ && opb == OB_ && acc == AC_)                                    \
    return launch_t<OA_, OB_, AC_>(M, N, K, A, lda, B, ldb, C, ldc, s);
  RBT_GEMM_CASE(OpA::General, OpB::General, Acc::SubtractTrailing)
  RBT_GEMM_CASE(OpA::GeneralT, OpB::General, Acc::Subtract)
  RBT_GEMM_CASE(OpA::General, OpB::Upper, Acc::Overwrite)
  RBT_GEMM_CASE(OpA::UnitLower, OpB::General, Acc::Overwrite)
  RBT_GEMM_CASE(OpA::Upper, OpB::General, Acc::Overwrite)
  RBT_GEMM_CASE(OpA::UnitLowerT, OpB::General, Acc::Overwrite)
  RBT_GEMM_CASE(OpA::UpperT, OpB::General, Acc::Overwrite)
#undef RBT_GEMM_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_dgemm_sub2(int64_t K, int64_t ld, int64_t M0, int64_t N0, const double *A0,
                             const double *B0, double *C0, int64_t M1, int64_t N1,
                             const double *A1, const double *B1, double *C1, hipStream_t s) {
  if (K <= 0) return hipSuccess;
  const int64_t t0 = M0 > 0 && N0 > 0 ? ((M0 + SM - 1) / SM) * ((N0 + SN - 1) / SN) : 0;
  const int64_t t1 = M1 > 0 && N1 > 0 ? ((M1 + SM - 1) / SM) * ((N1 + SN - 1) / SN) : 0;
  const int64_t start1 = (t0 + 7) / 8 * 8;
  if (start1 + t1 > 0x7fffffff) return hipErrorInvalidValue;
  if (start1 + t1 == 0) return hipSuccess;
  hipLaunchKernelGGL(k_dgemm_small2, dim3(unsigned(start1 + t1)), dim3(256), 0, s, K, ld,
                     sub_gemm(M0, N0, A0, B0, C0), sub_gemm(M1, N1, A1, B1, C1), int(start1));
  return hipGetLastError();
}

}  // namespace rbt
