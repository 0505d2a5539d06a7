// FP32-storage matrix-core GEMM for the mixed-precision elimination:
// C (M x N) -= A (M x K) B (K x N), column-major, all FP32 in memory.
//
//   kF32:  v_mfma_f32_16x16x4f32, FP32 operands and accumulation;
//   kBF16: operands rounded to BF16 (nearest even) when they are staged in
//          LDS, v_mfma_f32_16x16x32_bf16 (exact products, FP32
//          accumulation) -- the BF16 reading of the low-precision
//          factorization: BF16 update operands, FP32 accumulation and FP32
//          storage of the factors.
//
// Tiling: 256 threads = 4 wavefronts in a 2 x 2 grid, block tile 128 x 128,
// wavefront tile 64 x 64 = 4 x 4 MFMA tiles, K staged through LDS in slices
// of 32 with a register-prefetched double buffer (one barrier per slice).
// The depth-128 panel updates use 64 x 64 block tiles (k_sgemm_small).
// Both instructions leave output element (lane l, v) at row 4 (l / 16) + v,
// column l % 16 of their 16 x 16 tile (checked on the device), so a lane
// owns four consecutive rows of one column of C: the epilogue moves 16 bytes
// per lane.
//
// Operand layout in LDS: FP32 mode keeps A k-major (As[k][m]) and B n-major
// (Bs[n][k]); BF16 mode keeps both with k contiguous (8 BF16 = 16 bytes per
// lane and instruction). Block ids are remapped for the 8 XCDs and walked in
// groups of 8 tile rows, as in the FP64 GEMM.
#include "internal.h"

namespace rbt {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, BK = 32;
constexpr int GM = 8;
constexpr int kF32 = 0, kBF16 = 1;
// FP32 operand rows padded so that the lanes of one MFMA operand read hit
// distinct LDS banks: a row of As starts 16 banks after the previous one,
// a row of Bs 36 words after it (with 4 and 1, 40 % of the LDS cycles were
// bank conflicts; 2 % faster, identical results)
constexpr int PAD_AS = 16;  // As[k][BM + 16] (FP32)
constexpr int PAD_BS = 4;   // Bs[n][BK + 4] (FP32)
constexpr int PAD_H = 8;   // BF16 rows of BK + 8 (80 bytes)

template <int MODE>
struct Smem;
template <>
struct Smem<kF32> {
  alignas(16) float As[2][BK][BM + PAD_AS];
  alignas(16) float Bs[2][BN][BK + PAD_BS];
};
template <>
struct Smem<kBF16> {
  alignas(16) __bf16 Ah[2][BM][BK + PAD_H];
  alignas(16) __bf16 Bh[2][BN][BK + PAD_H];
};

// One 128 x 128 block tile at (m0, n0). FAST: an interior tile with K a
// multiple of BK (the kernel checks): unguarded loads in every slice and the
// whole-tile epilogue, with no per-slice branches between the matrix-core
// blocks. Every other tile takes the general body; both compute the same
// products in the same order.
template <int MODE, bool FAST>
__device__ __forceinline__ void sgemm_tile(int64_t M, int64_t N, int64_t K,
                                           const float *__restrict__ A, int64_t lda,
                                           const float *__restrict__ B, int64_t ldb, float *C,
                                           int64_t ldc, int64_t m0, int64_t n0, Smem<MODE> &sm) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int l16 = lane & 15, lk = lane >> 4;

  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};

  // staging coordinates
  //   FP32: A rows 4 (tid % 32) + 0..3 at k = tid / 32 + 8 p (16-byte loads),
  //   BF16: A row tid % 128 at k = 16 (tid / 128) + 0..15 (one 16-byte LDS
  //         store per 8 values: A is transposed to k-contiguous rows here);
  //   B (both): column tid / 2, k = 16 (tid % 2) + 4 p + 0..3.
  const int am = 4 * (tid & 31), ak = tid >> 5;
  const int hm = tid & (BM - 1), hk = 16 * (tid >> 7);
  const int bn = tid >> 1, bk = 16 * (tid & 1);
  f4 ra[4], rb[4];
  const bool interior = FAST || ((m0 + BM <= M) && (n0 + BN <= N));

  auto load_stage = [&](int64_t k0) {
    const bool fast = FAST || (interior && k0 + BK <= K);
    if constexpr (MODE == kF32) {
      if (fast) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const f4u v = *reinterpret_cast<const f4u *>(A + (m0 + am) + (k0 + ak + 8 * p) * lda);
          ra[p] = f4{v[0], v[1], v[2], v[3]};
        }
      } else {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const int64_t k = k0 + ak + 8 * p;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int64_t m = m0 + am + e;
            ra[p][e] = (m < M && k < K) ? A[m + k * lda] : 0.0f;
          }
        }
      }
    } else {
      const int64_t m = m0 + hm;
      if (fast) {
        const float *ap = A + m + (k0 + hk) * lda;
#pragma unroll
        for (int e = 0; e < 16; ++e) ra[e / 4][e % 4] = ap[e * lda];
      } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int64_t k = k0 + hk + e;
          ra[e / 4][e % 4] = (m < M && k < K) ? A[m + k * lda] : 0.0f;
        }
      }
    }
    if (fast) {
      const float *bp = B + (k0 + bk) + (n0 + bn) * ldb;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const f4u v = *reinterpret_cast<const f4u *>(bp + 4 * p);
        rb[p] = f4{v[0], v[1], v[2], v[3]};
      }
    } else {
      const int64_t n = n0 + bn;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t k = k0 + bk + 4 * p + e;
          rb[p][e] = (n < N && k < K) ? B[k + n * ldb] : 0.0f;
        }
      }
    }
  };

  auto store_stage = [&](int s) {
    if constexpr (MODE == kF32) {
#pragma unroll
      for (int p = 0; p < 4; ++p) *reinterpret_cast<f4 *>(&sm.As[s][ak + 8 * p][am]) = ra[p];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int e = 0; e < 4; ++e) sm.Bs[s][bn][bk + 4 * p + e] = rb[p][e];
    } else {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        bf8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (__bf16)ra[(8 * h + e) / 4][(8 * h + e) % 4];
        *reinterpret_cast<bf8 *>(&sm.Ah[s][hm][hk + 8 * h]) = v;
      }
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        bf4 v;
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (__bf16)rb[p][e];
        *reinterpret_cast<bf4 *>(&sm.Bh[s][bn][bk + 4 * p]) = v;
      }
    }
  };

  load_stage(0);
  store_stage(0);
  __syncthreads();

  int cur = 0;
  for (int64_t k0 = 0; k0 < K; k0 += BK) {
    const bool has_next = k0 + BK < K;
    if (has_next) load_stage(k0 + BK);
    if constexpr (MODE == kF32) {
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        float af[4], bf[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) af[i] = sm.As[cur][4 * kk + lk][wm * 64 + 16 * i + l16];
#pragma unroll
        for (int j = 0; j < 4; ++j) bf[j] = sm.Bs[cur][wn * 64 + 16 * j + l16][4 * kk + lk];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
    } else {
      bf8 af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        af[i] = *reinterpret_cast<const bf8 *>(&sm.Ah[cur][wm * 64 + 16 * i + l16][8 * lk]);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        bf[j] = *reinterpret_cast<const bf8 *>(&sm.Bh[cur][wn * 64 + 16 * j + l16][8 * lk]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    if (has_next) store_stage(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }

  // epilogue: acc[i][j][v] = (A B)[m0 + wm*64 + 16 i + 4 lk + v][n0 + wn*64 + 16 j + l16].
  // Whole tiles issue all 16 loads of C before the first store (a load of C
  // cannot be moved above a store to C by the compiler, which would
  // otherwise cost one round trip per load); edge tiles go element-wise.
  if (interior) {
    float *cp = C + (m0 + wm * 64 + 4 * lk) + (n0 + wn * 64 + l16) * ldc;
    f4u c[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        c[i][j] = *reinterpret_cast<const f4u *>(cp + 16 * i + 16 * j * ldc);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int v = 0; v < 4; ++v) c[i][j][v] -= acc[i][j][v];
        *reinterpret_cast<f4u *>(cp + 16 * i + 16 * j * ldc) = c[i][j];
      }
    return;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = m0 + wm * 64 + 16 * i + 4 * lk;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = n0 + wn * 64 + 16 * j + l16;
      if (col >= N) continue;
      float *p = C + row + col * ldc;
      if (row + 4 <= M) {
        f4u c = *reinterpret_cast<const f4u *>(p);
#pragma unroll
        for (int v = 0; v < 4; ++v) c[v] -= acc[i][j][v];
        *reinterpret_cast<f4u *>(p) = c;
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (row + v < M) p[v] -= acc[i][j][v];
      }
    }
  }
}

// WHOLE: every tile is interior and K a multiple of BK (the launcher
// checks); the kernel then holds only the fast tile body.
template <int MODE, bool TRAILING, bool WHOLE = false>
__global__ void __launch_bounds__(256, 2)
    k_sgemm(int64_t M, int64_t N, int64_t K, const float *__restrict__ A, int64_t lda,
            const float *__restrict__ B, int64_t ldb, float *C, int64_t ldc, int tiles_m,
            int total) {
  __shared__ Smem<MODE> sm;

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
  if (WHOLE || (m0 + BM <= M && n0 + BN <= N && K % BK == 0))
    sgemm_tile<MODE, true>(M, N, K, A, lda, B, ldb, C, ldc, m0, n0, sm);
  else if constexpr (!WHOLE)
    sgemm_tile<MODE, false>(M, N, K, A, lda, B, ldb, C, ldc, m0, n0, sm);
}

// Small tiles for the depth-128 updates inside and beside the panel (one
// dimension at most 896): 64 x 64 block tiles, 4 wavefronts of 32 x 32 (2 x 2
// MFMA tiles), K in slices of 32, 38 KB (FP32) / 20 KB (BF16) of LDS so that
// four workgroups share a CU. The same instructions over the same K order
// per output element as k_sgemm: identical results.
constexpr int SM = 64, SN = 64;

template <int MODE>
struct SmemS;
template <>
struct SmemS<kF32> {
  alignas(16) float As[2][BK][SM + PAD_AS];
  alignas(16) float Bs[2][SN][BK + PAD_BS];
};
template <>
struct SmemS<kBF16> {
  alignas(16) __bf16 Ah[2][SM][BK + PAD_H];
  alignas(16) __bf16 Bh[2][SN][BK + PAD_H];
};

// One 64 x 64 block tile; FAST as for the large tiles.
template <int MODE, bool FAST>
__device__ __forceinline__ void sgemm_small_tile(int64_t M, int64_t N, int64_t K,
                                                 const float *__restrict__ A, int64_t lda,
                                                 const float *__restrict__ B, int64_t ldb,
                                                 float *C, int64_t ldc, int64_t m0, int64_t n0,
                                                 SmemS<MODE> &sm) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int l16 = lane & 15, lk = lane >> 4;

  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};

  // staging coordinates
  //   FP32: A rows 4 (tid % 16) + 0..3 at k = tid / 16 + 16 p (16-byte loads),
  //   BF16: A row tid % 64 at k = 8 (tid / 64) + 0..7 (one 16-byte LDS store:
  //         A is transposed to k-contiguous rows here);
  //   B (both): column tid / 4, k = 8 (tid % 4) + 4 p + 0..3.
  const int am = 4 * (tid & 15), ak = tid >> 4;
  const int hm = tid & (SM - 1), hk = 8 * (tid >> 6);
  const int bn = tid >> 2, bk = 8 * (tid & 3);
  f4 ra[2], rb[2];
  const bool interior = FAST || ((m0 + SM <= M) && (n0 + SN <= N));

  auto load_stage = [&](int64_t k0) {
    const bool fast = FAST || (interior && k0 + BK <= K);
    if constexpr (MODE == kF32) {
      if (fast) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const f4u v = *reinterpret_cast<const f4u *>(A + (m0 + am) + (k0 + ak + 16 * p) * lda);
          ra[p] = f4{v[0], v[1], v[2], v[3]};
        }
      } else {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const int64_t k = k0 + ak + 16 * p;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int64_t m = m0 + am + e;
            ra[p][e] = (m < M && k < K) ? A[m + k * lda] : 0.0f;
          }
        }
      }
    } else {
      const int64_t m = m0 + hm;
      if (fast) {
        const float *ap = A + m + (k0 + hk) * lda;
#pragma unroll
        for (int e = 0; e < 8; ++e) ra[e / 4][e % 4] = ap[e * lda];
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int64_t k = k0 + hk + e;
          ra[e / 4][e % 4] = (m < M && k < K) ? A[m + k * lda] : 0.0f;
        }
      }
    }
    if (fast) {
      const float *bp = B + (k0 + bk) + (n0 + bn) * ldb;
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const f4u v = *reinterpret_cast<const f4u *>(bp + 4 * p);
        rb[p] = f4{v[0], v[1], v[2], v[3]};
      }
    } else {
      const int64_t n = n0 + bn;
#pragma unroll
      for (int p = 0; p < 2; ++p) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t k = k0 + bk + 4 * p + e;
          rb[p][e] = (n < N && k < K) ? B[k + n * ldb] : 0.0f;
        }
      }
    }
  };

  auto store_stage = [&](int s) {
    if constexpr (MODE == kF32) {
#pragma unroll
      for (int p = 0; p < 2; ++p) *reinterpret_cast<f4 *>(&sm.As[s][ak + 16 * p][am]) = ra[p];
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int e = 0; e < 4; ++e) sm.Bs[s][bn][bk + 4 * p + e] = rb[p][e];
    } else {
      bf8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (__bf16)ra[e / 4][e % 4];
      *reinterpret_cast<bf8 *>(&sm.Ah[s][hm][hk]) = v;
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        bf4 w;
#pragma unroll
        for (int e = 0; e < 4; ++e) w[e] = (__bf16)rb[p][e];
        *reinterpret_cast<bf4 *>(&sm.Bh[s][bn][bk + 4 * p]) = w;
      }
    }
  };

  load_stage(0);
  store_stage(0);
  __syncthreads();

  int cur = 0;
  for (int64_t k0 = 0; k0 < K; k0 += BK) {
    const bool has_next = k0 + BK < K;
    if (has_next) load_stage(k0 + BK);
    if constexpr (MODE == kF32) {
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        float af[2], bf[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) af[i] = sm.As[cur][4 * kk + lk][wm * 32 + 16 * i + l16];
#pragma unroll
        for (int j = 0; j < 2; ++j) bf[j] = sm.Bs[cur][wn * 32 + 16 * j + l16][4 * kk + lk];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
    } else {
      bf8 af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        af[i] = *reinterpret_cast<const bf8 *>(&sm.Ah[cur][wm * 32 + 16 * i + l16][8 * lk]);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        bf[j] = *reinterpret_cast<const bf8 *>(&sm.Bh[cur][wn * 32 + 16 * j + l16][8 * lk]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    if (has_next) store_stage(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }

  // epilogue: acc[i][j][v] = (A B)[m0 + wm*32 + 16 i + 4 lk + v][n0 + wn*32 + 16 j + l16]
  if (interior) {
    float *cp = C + (m0 + wm * 32 + 4 * lk) + (n0 + wn * 32 + l16) * ldc;
    f4u c[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) c[i][j] = *reinterpret_cast<const f4u *>(cp + 16 * i + 16 * j * ldc);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int v = 0; v < 4; ++v) c[i][j][v] -= acc[i][j][v];
        *reinterpret_cast<f4u *>(cp + 16 * i + 16 * j * ldc) = c[i][j];
      }
    return;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int64_t row = m0 + wm * 32 + 16 * i + 4 * lk;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t col = n0 + wn * 32 + 16 * j + l16;
      if (col >= N) continue;
      float *p = C + row + col * ldc;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (row + v < M) p[v] -= acc[i][j][v];
    }
  }
}

template <int MODE>
__global__ void __launch_bounds__(256, 4)
    k_sgemm_small(int64_t M, int64_t N, int64_t K, const float *__restrict__ A, int64_t lda,
                  const float *__restrict__ B, int64_t ldb, float *C, int64_t ldc, int tiles_m,
                  int total) {
  __shared__ SmemS<MODE> sm;

  int pid = blockIdx.x;
  const int full = (total / 8) * 8;
  if (pid < full) pid = (pid % 8) * (total / 8) + pid / 8;
  const int tiles_n = total / tiles_m;
  const int group = pid / (GM * tiles_n);
  const int first_m = group * GM;
  const int gsize = (tiles_m - first_m) < GM ? (tiles_m - first_m) : GM;
  const int in_group = pid - group * GM * tiles_n;
  const int tm = first_m + in_group % gsize, tn = in_group / gsize;
  const int64_t m0 = int64_t(tm) * SM, n0 = int64_t(tn) * SN;
  if (m0 + SM <= M && n0 + SN <= N && K % BK == 0)
    sgemm_small_tile<MODE, true>(M, N, K, A, lda, B, ldb, C, ldc, m0, n0, sm);
  else
    sgemm_small_tile<MODE, false>(M, N, K, A, lda, B, ldb, C, ldc, m0, n0, sm);
}

template <int MODE>
hipError_t launch_small(int64_t M, int64_t N, int64_t K, const float *A, int64_t lda,
                        const float *B, int64_t ldb, float *C, int64_t ldc, hipStream_t s) {
  const int64_t tm = (M + SM - 1) / SM, tn = (N + SN - 1) / SN;
  const int64_t total = tm * tn;
  if (total > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_sgemm_small<MODE>), dim3(unsigned(total)), dim3(256), 0, s, M, N, K, A,
                     lda, B, ldb, C, ldc, int(tm), int(total));
  return hipGetLastError();
}

template <int MODE, bool TRAILING>
hipError_t launch_t(int64_t M, int64_t N, int64_t K, const float *A, int64_t lda, const float *B,
                    int64_t ldb, float *C, int64_t ldc, hipStream_t s) {
  const int64_t tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN;
  const int64_t total = tm * tn;
  if (total > 0x7fffffff) return hipErrorInvalidValue;
  if constexpr (TRAILING) {
    if (M % BM == 0 && N % BN == 0 && K % BK == 0) {
      hipLaunchKernelGGL((k_sgemm<MODE, TRAILING, true>), dim3(unsigned(total)), dim3(256), 0, s,
                         M, N, K, A, lda, B, ldb, C, ldc, int(tm), int(total));
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_sgemm<MODE, TRAILING>), dim3(unsigned(total)), dim3(256), 0, s, M, N, K,
                     A, lda, B, ldb, C, ldc, int(tm), int(total));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_sgemm_sub(int64_t M, int64_t N, int64_t K, const float *A, int64_t lda,
                            const float *B, int64_t ldb, float *C, int64_t ldc, bool bf16,
                            bool trailing, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  // the trailing update on the large tiles, the panel and block-row updates
  // on the small ones (with BF16 operands the block rows, M < N, were as
  // fast on the large tiles at depth 128; with the deeper updates of the
  // recursive panel order the small tiles are 0.6 % faster per solve)
  if (bf16) {
    if (trailing) return launch_t<kBF16, true>(M, N, K, A, lda, B, ldb, C, ldc, s);
    return launch_small<kBF16>(M, N, K, A, lda, B, ldb, C, ldc, s);
  }
  return trailing ? launch_t<kF32, true>(M, N, K, A, lda, B, ldb, C, ldc, s)
                  : launch_small<kF32>(M, N, K, A, lda, B, ldb, C, ldc, s);
}

hipError_t launch_sgemm_tiles(int tile, int64_t M, int64_t N, int64_t K, const float *A,
                              int64_t lda, const float *B, int64_t ldb, float *C, int64_t ldc,
                              bool bf16, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  if (tile == 64)
    return bf16 ? launch_small<kBF16>(M, N, K, A, lda, B, ldb, C, ldc, s)
                : launch_small<kF32>(M, N, K, A, lda, B, ldb, C, ldc, s);
  return bf16 ? launch_t<kBF16, false>(M, N, K, A, lda, B, ldb, C, ldc, s)
              : launch_t<kF32, false>(M, N, K, A, lda, B, ldb, C, ldc, s);
}

}  // namespace rbt
