// Trailing update of the BF16-operand elimination, C (FP32, M x N) -= L21 U12,
// with the operands rounded to BF16 once per update instead of once per tile.
//
// The FP32 factors are kept in FP32 (the BF16 reading of the low-precision
// elimination: BF16 update operands, FP32 accumulation and storage). For a
// trailing update the panel L21 (M x K) and the block row U12 (K x N) are
// first rounded to BF16 (nearest even) into k-contiguous staging buffers:
//   Lb[m][k]  (row-major, rows padded with zeros to whole 256-row tiles),
//   Ub[n][k]  (column-major, columns padded with zeros likewise),
// 2 bytes per element instead of the 4 that every tile would otherwise fetch
// and convert. The GEMM then runs 256 x 256 tiles with 8 wavefronts (2 x 4,
// 128 x 64 each = 8 x 4 tiles of v_mfma_f32_16x16x32_bf16), K staged through
// LDS in slices of 64, double-buffered, loads two slices ahead. Per slice a
// workgroup reads 64 KB for 8.4 MFLOP: four times the arithmetic intensity
// of the 128 x 128 FP32-operand tile.
//
// Every output element accumulates the same BF16 products in the same order
// (K in steps of 32, lane l supplying k = 8 (l / 16) + 0..7 of a step) as
// the FP32-storage GEMM in BF16 mode, so the results are identical.
// Output element (lane l, v) of the instruction is row 4 (l / 16) + v,
// column l % 16 of its 16 x 16 tile (checked on the device): the epilogue
// reads and writes 16 bytes per lane.
#include "internal.h"

namespace rbt {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

constexpr int HM = 256, HN = 256, HK = 64;
// LDS rows of HK = 64 BF16 (128 bytes, eight 16-byte chunks). Chunk q of
// row r is stored at position q ^ (r & 7): the 16 lanes that read one
// k-chunk of 16 consecutive rows then spread over all positions (with
// padded 144-byte rows 37 % of the LDS cycles were bank conflicts; the
// swizzle is 5 % faster at 16384^2 x 1024 and bit-identical).
constexpr int HLD = HK;
constexpr int GM = 8;        // tile rows per ordering group

// Lb[m * Kp + k] = bf16(L[m + k * ldl]) for m < M, zero for M <= m < Mp.
// Thread: one row m, 8 consecutive k (one 16-byte store); consecutive
// threads take consecutive rows, so the FP32 reads are coalesced.
__global__ void __launch_bounds__(256) k_cvt_rows(int64_t M, int64_t Mp, int64_t K,
                                                  const float *__restrict__ L, int64_t ldl,
                                                  __bf16 *__restrict__ Lb) {
  const int64_t m = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int64_t k0 = int64_t(blockIdx.y) * 8;
  if (m >= Mp) return;
  bf8 v;
  const int64_t mc = m < M ? m : M - 1;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float x = L[mc + (k0 + e) * ldl];
    v[e] = m < M ? (__bf16)x : (__bf16)0.0f;
  }
  *reinterpret_cast<bf8 *>(Lb + m * K + k0) = v;
}

// Ub[n * K + k] = bf16(U[k + n * ldu]) for n < N, zero for N <= n < Np.
__global__ void __launch_bounds__(256) k_cvt_cols(int64_t N, int64_t Np, int64_t K,
                                                  const float *__restrict__ U, int64_t ldu,
                                                  __bf16 *__restrict__ Ub) {
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;  // (n, chunk of 8 k)
  const int64_t chunks = K / 8;
  const int64_t n = idx / chunks, k0 = (idx % chunks) * 8;
  if (n >= Np) return;
  bf8 v;
  const int64_t nc = n < N ? n : N - 1;
  const float *p = U + k0 + nc * ldu;
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = n < N ? (__bf16)p[e] : (__bf16)0.0f;
  *reinterpret_cast<bf8 *>(Ub + n * K + k0) = v;
}

__global__ void __launch_bounds__(512, 1)
    k_hgemm(int64_t M, int64_t N, int64_t K, const __bf16 *__restrict__ Lb,
            const __bf16 *__restrict__ Ub, float *C, int64_t ldc, int tiles_m, int total) {
  __shared__ __attribute__((aligned(16))) __bf16 As[2][HM][HLD];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][HN][HLD];

  // XCD-aware remap, then grouped tile order (as the other GEMMs)
  int pid = blockIdx.x;
  const int full = (total / 8) * 8;
  if (pid < full) pid = (pid % 8) * (total / 8) + pid / 8;
  const int tiles_n = total / tiles_m;
  const int group = pid / (GM * tiles_n);
  const int first_m = group * GM;
  const int gsize = (tiles_m - first_m) < GM ? (tiles_m - first_m) : GM;
  const int in_group = pid - group * GM * tiles_n;
  const int tm = first_m + in_group % gsize, tn = in_group / gsize;
  const int64_t m0 = int64_t(tm) * HM, n0 = int64_t(tn) * HN;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;  // 2 x 4 wavefronts: 128 rows x 64 columns each
  const int l16 = lane & 15, lk = lane >> 4;

  f4 acc[8][4];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};

  // staging: 2048 chunks of 16 bytes per operand and slice, 4 per thread:
  // chunk c = tid + 512 p -> tile row (or column) c / 8, k = 8 (c % 8)
  u4 ra[4], rb[4];
  const __bf16 *pa = Lb + m0 * K;
  const __bf16 *pb = Ub + n0 * K;
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int c = tid + 512 * p;
      const int64_t off = int64_t(c >> 3) * K + k0 + 8 * (c & 7);
      ra[p] = *reinterpret_cast<const u4 *>(pa + off);
      rb[p] = *reinterpret_cast<const u4 *>(pb + off);
    }
  };
  auto store = [&](int s) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int c = tid + 512 * p;
      const int row = c >> 3, q = (c & 7) ^ (row & 7);
      *reinterpret_cast<u4 *>(&As[s][row][8 * q]) = ra[p];
      *reinterpret_cast<u4 *>(&Bs[s][row][8 * q]) = rb[p];
    }
  };

  // slice s is multiplied from LDS buffer s % 2 while slice s + 1 goes from
  // registers into the other buffer (free since the barrier that ended slice
  // s - 1) and the loads of slice s + 2 are in flight
  load(0);
  store(0);
  if (HK < K) load(HK);
  __syncthreads();
  int cur = 0;
  for (int64_t k0 = 0; k0 < K; k0 += HK) {
    if (k0 + HK < K) {
      store(cur ^ 1);
      if (k0 + 2 * HK < K) load(k0 + 2 * HK);
    }
#pragma unroll
    for (int kk = 0; kk < HK / 32; ++kk) {
      bf8 a[8], b[4];
#pragma unroll
      for (int i = 0; i < 8; ++i)
        a[i] = *reinterpret_cast<const bf8 *>(
            &As[cur][wm * 128 + 16 * i + l16][8 * ((4 * kk + lk) ^ (l16 & 7))]);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        b[j] = *reinterpret_cast<const bf8 *>(
            &Bs[cur][wn * 64 + 16 * j + l16][8 * ((4 * kk + lk) ^ (l16 & 7))]);
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
    cur ^= 1;
  }

  // epilogue: acc[i][j][v] = (L21 U12)[m0 + wm*128 + 16 i + 4 lk + v][n0 + wn*64 + 16 j + l16].
  // Whole tiles keep the loads of C two row blocks ahead of the stores (a
  // load of C cannot be moved above a store to C by the compiler, which
  // would otherwise cost one round trip per load); edge tiles go one by one.
  if (m0 + HM <= M && n0 + HN <= N) {
    float *cp = C + (m0 + wm * 128 + 4 * lk) + (n0 + wn * 64 + l16) * ldc;
    f4u c[3][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) c[i][j] = *reinterpret_cast<const f4u *>(cp + 16 * i + 16 * j * ldc);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (i + 2 < 8) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          c[(i + 2) % 3][j] = *reinterpret_cast<const f4u *>(cp + 16 * (i + 2) + 16 * j * ldc);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        f4u r = c[i % 3][j];
#pragma unroll
        for (int v = 0; v < 4; ++v) r[v] -= acc[i][j][v];
        *reinterpret_cast<f4u *>(cp + 16 * i + 16 * j * ldc) = r;
      }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int64_t row = m0 + wm * 128 + 16 * i + 4 * lk;
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

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

}  // namespace

size_t hgemm_stage_bytes(int64_t M, int64_t N, int64_t K) {
  if (M <= 0 || N <= 0 || K <= 0) return 0;
  return size_t(round_up(M, HM) + round_up(N, HN)) * size_t(K) * sizeof(__bf16) + 256;
}

bool hgemm_supported(int64_t K) { return K > 0 && K % HK == 0; }

hipError_t launch_hgemm_sub(int64_t M, int64_t N, int64_t K, const float *L21, int64_t ldl,
                            const float *U12, int64_t ldu, float *C, int64_t ldc, void *stage,
                            size_t stage_bytes, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  if (!hgemm_supported(K) || stage == nullptr || stage_bytes < hgemm_stage_bytes(M, N, K))
    return hipErrorInvalidValue;
  const int64_t Mp = round_up(M, HM), Np = round_up(N, HN);
  const int64_t tm = Mp / HM, tn = Np / HN, total = tm * tn;
  if (total > 0x7fffffff || Mp / 256 > 0x7fffffff || K / 8 > 65535) return hipErrorInvalidValue;
  char *base = static_cast<char *>(stage);
  base += (256 - (reinterpret_cast<uintptr_t>(base) & 255)) & 255;  // 256-byte alignment
  __bf16 *Lb = reinterpret_cast<__bf16 *>(base);
  __bf16 *Ub = Lb + Mp * K;
  hipLaunchKernelGGL(k_cvt_rows, dim3(unsigned(Mp / 256), unsigned(K / 8)), dim3(256), 0, s, M,
                     Mp, K, L21, ldl, Lb);
  const int64_t cvt_threads = Np * (K / 8);
  hipLaunchKernelGGL(k_cvt_cols, dim3(unsigned((cvt_threads + 255) / 256)), dim3(256), 0, s, N,
                     Np, K, U12, ldu, Ub);
  hipLaunchKernelGGL(k_hgemm, dim3(unsigned(total)), dim3(512), 0, s, M, N, K, Lb, Ub, C, ldc,
                     int(tm), int(total));
  return hipGetLastError();
}

}  // namespace rbt
