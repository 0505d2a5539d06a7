// Block triangular solves with a factored kb x kb diagonal block (kb <= 128)
// of the elimination, 16 rows (columns) at a time: the update from the
// blocks already solved runs on the FP64 matrix cores, and each 16 x 16
// diagonal block is solved by plain substitution (one lane per right-hand
// side), so the rounding behaviour is that of ordinary forward/back
// substitution except that a division by a pivot is a multiplication by its
// reciprocal (within one rounding of the quotient). (Multiplying by explicit
// inverses of the diagonal blocks, even 16 x 16 ones, raised the backward
// error several-fold on N(0,1) matrices with large growth.)
//
// LDS holds the right-hand-side strips and the eight 16 x 16 diagonal blocks
// (80 KB, two workgroups per CU); the off-diagonal operands of each step are
// loaded from global memory into registers while the previous step's
// barrier and substitution run.
//
// Left solves, op(T) X = B in place (B: kb x N):
//   LN  T = L (unit lower)     forward  (panel U12 = L11^-1 A12, L y = b)
//   UN  T = U (upper)          backward (U x = y)
//   UT  T = U^T (lower)        forward  (U^T z = g, adjoint solves)
//   LT  T = L^T (unit upper)   backward (L^T w = z)
//   X_I = T_II \ (B_I - sum_{J before I} T_IJ X_J)
// Each wavefront owns 16 columns of B; a workgroup of four covers 64.
//
// Right solve, X U = B in place (B: M x kb) for the panel L21 = A21 U11^-1:
//   X_J = (B_J - sum_{I<J} X_I U_IJ) / U_JJ
// Each wavefront owns 16 rows of B.
//
// MFMA: v_mfma_f64_16x16x4_f64 with the standard operand order; its output
// element (lane l, v) is row l/16 + 4v, column l % 16.
//
// The triangle (TT) and the right-hand sides (TB) may be stored in FP32
// (mixed-precision elimination); values are widened on load and all
// arithmetic is FP64, rounded once on store.
#include "internal.h"

namespace rbt {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int NB = kNB;  // 128
constexpr int IB = 16;
constexpr int NBK = NB / IB;  // 8 diagonal blocks
constexpr int BLK = IB * IB;  // 256 doubles per block

template <TriMode MODE>
constexpr bool forward_order() {
  return MODE == TriMode::LN || MODE == TriMode::UT;
}
template <TriMode MODE>
constexpr bool unit_diag() {
  return MODE == TriMode::LN || MODE == TriMode::LT;
}

// op(T)(i, j) read from global memory (i, j < kb), in the stored type.
// Loads are issued unconditionally at clamped valid indices and masked
// afterwards, so that a batch of them is in flight together (a conditional
// load per element, or a widening right after it, serializes them).
template <TriMode MODE, typename TT>
__device__ __forceinline__ TT op_t(const TT *T, int64_t ldt, int i, int j) {
  if constexpr (MODE == TriMode::LN || MODE == TriMode::UN)
    return T[i + int64_t(j) * ldt];
  else
    return T[j + int64_t(i) * ldt];
}
__device__ __forceinline__ int clampi(int v, int hi) { return v < hi ? v : hi; }

// BATCH: blockIdx.y selects diagonal block b of an n x n factor (T and B
// offset by b * kNB (1 + ldt) and b * bstride, kb = min(kNB, n - b kNB)), and
// the right-hand side is the identity (X = op(T_bb)^-1): used to form the
// inverses of the diagonal blocks once per factorization.
template <TriMode MODE, bool BATCH, typename TT, typename TB>
__global__ void __launch_bounds__(256, 2) k_trsm_left(int kb, int64_t N, const TT *T,
                                                      int64_t ldt, TB *B, int64_t ldb,
                                                      int64_t n, int64_t bstride) {
  if constexpr (BATCH) {
    const int64_t b = blockIdx.y;
    const int64_t r0 = b * NB;
    kb = int(n - r0 < NB ? n - r0 : NB);
    N = kb;
    T += r0 + r0 * ldt;
    B += b * bstride;
  }
  __shared__ double dblk[NBK * BLK];        // diagonal blocks of op(T), element (i,j) at j*16+i
  __shared__ double strip_all[4][NB * IB];  // per wavefront: row-major 128 x 16
  constexpr bool FWD = forward_order<MODE>();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  double *strip = strip_all[wave];
  const int64_t col0 = int64_t(blockIdx.x) * 64 + wave * 16;

  {  // stage the diagonal blocks (reciprocal on the diagonal of non-unit modes)
    const int i = threadIdx.x % IB, j = threadIdx.x / IB;
    TT raw[NBK];
#pragma unroll
    for (int b = 0; b < NBK; ++b)
      raw[b] = op_t<MODE>(T, ldt, clampi(IB * b + i, kb - 1), clampi(IB * b + j, kb - 1));
#pragma unroll
    for (int b = 0; b < NBK; ++b) {
      const int gi = IB * b + i, gj = IB * b + j;
      double v = (gi < kb && gj < kb) ? double(raw[b]) : (i == j ? 1.0 : 0.0);
      if (!unit_diag<MODE>() && i == j) v = 1.0 / v;
      dblk[b * BLK + j * IB + i] = v;
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {  // strip: lane = row (two halves), 16 columns
    const int row = lane + 64 * h;
    if constexpr (BATCH) {
#pragma unroll
      for (int c = 0; c < IB; ++c) {
        const int64_t col = col0 + c;
        strip[row * IB + c] = (row < kb && col < N && row == col) ? 1.0 : 0.0;
      }
    } else {
      TB raw[IB];
      const int64_t rr = clampi(row, kb - 1);
#pragma unroll
      for (int c = 0; c < IB; ++c) {
        const int64_t col = col0 + c < N ? col0 + c : N - 1;
        raw[c] = B[rr + col * ldb];
      }
#pragma unroll
      for (int c = 0; c < IB; ++c)
        strip[row * IB + c] = (row < kb && col0 + c < N) ? double(raw[c]) : 0.0;
    }
  }
  __syncthreads();

  const int nbk = (kb + IB - 1) / IB;
  // off-diagonal operands of a step, op(T)[16 I + l16][16 J + 4 kk + lk];
  // those of step + 1 are loaded once the MFMAs of step have consumed these,
  // so the loads are in flight during the barrier and the substitution
  TT araw[NBK - 1][4];
  auto load_step = [&](int st) {
    const int ia = IB * (FWD ? st : nbk - 1 - st) + l16;
#pragma unroll
    for (int s2 = 0; s2 < NBK - 1; ++s2) {
      const int J = FWD ? s2 : nbk - 1 - s2;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int kx = IB * J + 4 * kk + lk;
        araw[s2][kk] = op_t<MODE>(T, ldt, clampi(ia, kb - 1), clampi(kx < 0 ? 0 : kx, kb - 1));
      }
    }
  };
  load_step(0);
  for (int step = 0; step < nbk; ++step) {
    const int I = FWD ? step : nbk - 1 - step;
    const int ia = IB * I + l16;
    double a[NBK - 1][4];
#pragma unroll
    for (int s2 = 0; s2 < NBK - 1; ++s2) {
      const int J = FWD ? s2 : nbk - 1 - s2;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int kx = IB * J + 4 * kk + lk;
        a[s2][kk] = (s2 < step && ia < kb && kx >= 0 && kx < kb) ? double(araw[s2][kk]) : 0.0;
      }
    }
    d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s2 = 0; s2 < NBK - 1; ++s2) {
      if (s2 < step) {
        const int J = FWD ? s2 : nbk - 1 - s2;
        const int k0 = IB * J + lk;
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s2][0], strip[(k0) * IB + l16], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s2][1], strip[(k0 + 4) * IB + l16], acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s2][2], strip[(k0 + 8) * IB + l16], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s2][3], strip[(k0 + 12) * IB + l16], acc1, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) strip[(IB * I + lk + 4 * v) * IB + l16] -= acc0[v] + acc1[v];
    if (step + 1 < nbk) load_step(step + 1);
    __syncthreads();
    // substitution inside the diagonal block: lane c < 16 owns column c
    const int bs = kb - IB * I < IB ? kb - IB * I : IB;
    if (lane < IB) {
      const int o = IB * I;
      const double *tb = dblk + I * BLK;
      double x[IB];
#pragma unroll
      for (int i = 0; i < IB; ++i) x[i] = strip[(o + i) * IB + lane];
      if constexpr (FWD) {
#pragma unroll
        for (int j = 0; j < IB; ++j) {
          if (j < bs) {
            if constexpr (!unit_diag<MODE>()) x[j] *= tb[j * IB + j];
#pragma unroll
            for (int i = j + 1; i < IB; ++i) x[i] -= tb[j * IB + i] * x[j];
          }
        }
      } else {
#pragma unroll
        for (int j = IB - 1; j >= 0; --j) {
          if (j < bs) {
            if constexpr (!unit_diag<MODE>()) x[j] *= tb[j * IB + j];
#pragma unroll
            for (int i = 0; i < j; ++i) x[i] -= tb[j * IB + i] * x[j];
          }
        }
      }
#pragma unroll
      for (int i = 0; i < IB; ++i) strip[(o + i) * IB + lane] = (i < bs) ? x[i] : 0.0;
    }
    __syncthreads();
  }

#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int row = lane + 64 * h;
#pragma unroll
    for (int c = 0; c < IB; ++c) {
      const int64_t col = col0 + c;
      if (row < kb && col < N) B[row + col * ldb] = TB(strip[row * IB + c]);
    }
  }
}

template <typename TT>
__global__ void __launch_bounds__(256, 2) k_trsm_right_upper(int kb, int64_t M, const TT *T,
                                                             int64_t ldt, TT *B,
                                                             int64_t ldb) {
  __shared__ double dblk[NBK * BLK];        // diagonal blocks of U, element (r,c) at r*16+c
  __shared__ double strip_all[4][NB * IB];  // per wavefront: column-major 16 x 128
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  double *strip = strip_all[wave];
  const int64_t row0 = int64_t(blockIdx.x) * 64 + wave * 16;

  {
    const int r = threadIdx.x % IB, c = threadIdx.x / IB;
    TT raw[NBK];
#pragma unroll
    for (int b = 0; b < NBK; ++b)
      raw[b] = T[clampi(IB * b + r, kb - 1) + int64_t(clampi(IB * b + c, kb - 1)) * ldt];
#pragma unroll
    for (int b = 0; b < NBK; ++b) {
      const int gi = IB * b + r, gj = IB * b + c;
      double v = (gi < kb && gj < kb) ? double(raw[b]) : (r == c ? 1.0 : 0.0);
      if (r == c) v = 1.0 / v;
      dblk[b * BLK + r * IB + c] = v;
    }
  }
  {
    // lane = (row r = lane % 16, column group lane / 16): columns cg + 4u
    const int r = lane % IB, cg = lane / IB;
    const int64_t row = row0 + r;
    const int64_t rr = row < M ? row : M - 1;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      TT raw[16];
#pragma unroll
      for (int u = 0; u < 16; ++u)
        raw[u] = B[rr + int64_t(clampi(cg + 4 * (16 * h + u), kb - 1)) * ldb];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int c = cg + 4 * (16 * h + u);
        strip[c * IB + r] = (row < M && c < kb) ? double(raw[u]) : 0.0;
      }
    }
  }
  __syncthreads();

  const int nbk = (kb + IB - 1) / IB;
  // off-diagonal operands of step J, U[16 I + 4 kk + lk][16 J + l16]; those
  // of J + 1 are loaded once the MFMAs of J have consumed these
  TT braw[NBK - 1][4];
  auto load_step = [&](int st) {
    const int jc = IB * st + l16;
#pragma unroll
    for (int I = 0; I < NBK - 1; ++I) {
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
        braw[I][kk] = T[clampi(IB * I + 4 * kk + lk, kb - 1) + int64_t(clampi(jc, kb - 1)) * ldt];
    }
  };
  load_step(0);
  for (int J = 0; J < nbk; ++J) {
    const int jc = IB * J + l16;  // column of U this lane feeds
    double b[NBK - 1][4];
#pragma unroll
    for (int I = 0; I < NBK - 1; ++I) {
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int kx = IB * I + 4 * kk + lk;
        b[I][kk] = (I < J && kx < kb && jc < kb) ? double(braw[I][kk]) : 0.0;
      }
    }
    d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int I = 0; I < NBK - 1; ++I) {
      if (I < J) {
        const int k0 = IB * I + lk;
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(strip[(k0) * IB + l16], b[I][0], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(strip[(k0 + 4) * IB + l16], b[I][1], acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(strip[(k0 + 8) * IB + l16], b[I][2], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(strip[(k0 + 12) * IB + l16], b[I][3], acc1, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) strip[(IB * J + l16) * IB + lk + 4 * v] -= acc0[v] + acc1[v];
    if (J + 1 < nbk) load_step(J + 1);
    __syncthreads();
    // substitution inside the diagonal block: lane r < 16 owns row r
    const int bs = kb - IB * J < IB ? kb - IB * J : IB;
    if (lane < IB) {
      const int o = IB * J;
      const double *tb = dblk + J * BLK;
      double x[IB];
#pragma unroll
      for (int c = 0; c < IB; ++c) x[c] = strip[(o + c) * IB + lane];
#pragma unroll
      for (int c = 0; c < IB; ++c) {
        if (c < bs) {
          x[c] *= tb[c * IB + c];
#pragma unroll
          for (int c2 = c + 1; c2 < IB; ++c2) x[c2] -= x[c] * tb[c * IB + c2];
        }
      }
#pragma unroll
      for (int c = 0; c < IB; ++c) strip[(o + c) * IB + lane] = (c < bs) ? x[c] : 0.0;
    }
    __syncthreads();
  }

  {
    const int r = lane % IB, cg = lane / IB;
    const int64_t row = row0 + r;
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const int c = cg + 4 * u;
      if (row < M && c < kb) B[row + int64_t(c) * ldb] = TT(strip[c * IB + r]);
    }
  }
}

template <typename TT, typename TB>
hipError_t trsm_left_t(TriMode mode, int kb, int64_t N, const TT *T, int64_t ldt, TB *B,
                       int64_t ldb, hipStream_t s) {
  if (kb <= 0 || N <= 0) return hipSuccess;
  if (kb > kNB) return hipErrorInvalidValue;
  const dim3 grid(unsigned((N + 63) / 64));
  const int64_t z = 0;
  switch (mode) {
    case TriMode::LN: hipLaunchKernelGGL((k_trsm_left<TriMode::LN, false, TT, TB>), grid, dim3(256), 0, s, kb, N, T, ldt, B, ldb, z, z); break;
    case TriMode::UN: hipLaunchKernelGGL((k_trsm_left<TriMode::UN, false, TT, TB>), grid, dim3(256), 0, s, kb, N, T, ldt, B, ldb, z, z); break;
    case TriMode::UT: hipLaunchKernelGGL((k_trsm_left<TriMode::UT, false, TT, TB>), grid, dim3(256), 0, s, kb, N, T, ldt, B, ldb, z, z); break;
    case TriMode::LT: hipLaunchKernelGGL((k_trsm_left<TriMode::LT, false, TT, TB>), grid, dim3(256), 0, s, kb, N, T, ldt, B, ldb, z, z); break;
  }
  return hipGetLastError();
}

template <typename TT>
hipError_t diag_inverses_t(int64_t n, const TT *LU, int64_t ld, double *W, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + NB - 1) / NB;
  if (nb > 65535) return hipErrorInvalidValue;
  const dim3 grid(2, unsigned(nb));  // 2 x 64 columns of each 128 x 128 block
  // L^-1 at W + b * 2 kNB^2, U^-1 at W + b * 2 kNB^2 + kNB^2, each ld kNB
  hipLaunchKernelGGL((k_trsm_left<TriMode::LN, true, TT, double>), grid, dim3(256), 0, s, NB,
                     int64_t(NB), LU, ld, W, int64_t(NB), n, int64_t(2 * NB * NB));
  hipLaunchKernelGGL((k_trsm_left<TriMode::UN, true, TT, double>), grid, dim3(256), 0, s, NB,
                     int64_t(NB), LU, ld, W + NB * NB, int64_t(NB), n, int64_t(2 * NB * NB));
  return hipGetLastError();
}

template <typename TT>
hipError_t trsm_right_upper_t(int kb, int64_t M, const TT *T, int64_t ldt, TT *B, int64_t ldb,
                              hipStream_t s) {
  if (kb <= 0 || M <= 0) return hipSuccess;
  if (kb > kNB) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_trsm_right_upper<TT>, dim3(unsigned((M + 63) / 64)), dim3(256), 0, s, kb,
                     M, T, ldt, B, ldb);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_trsm_left(TriMode mode, int kb, int64_t N, const double *T, int64_t ldt,
                            double *B, int64_t ldb, hipStream_t s) {
  return trsm_left_t(mode, kb, N, T, ldt, B, ldb, s);
}
hipError_t launch_trsm_left(TriMode mode, int kb, int64_t N, const float *T, int64_t ldt, float *B,
                            int64_t ldb, hipStream_t s) {
  return trsm_left_t(mode, kb, N, T, ldt, B, ldb, s);
}
hipError_t launch_diag_inverses(int64_t n, const double *LU, int64_t ld, double *W,
                                hipStream_t s) {
  return diag_inverses_t(n, LU, ld, W, s);
}
hipError_t launch_diag_inverses(int64_t n, const float *LU, int64_t ld, double *W, hipStream_t s) {
  return diag_inverses_t(n, LU, ld, W, s);
}
hipError_t launch_trsm_right_upper(int kb, int64_t M, const double *T, int64_t ldt, double *B,
                                   int64_t ldb, hipStream_t s) {
  return trsm_right_upper_t(kb, M, T, ldt, B, ldb, s);
}
hipError_t launch_trsm_right_upper(int kb, int64_t M, const float *T, int64_t ldt, float *B,
                                   int64_t ldb, hipStream_t s) {
  return trsm_right_upper_t(kb, M, T, ldt, B, ldb, s);
}

}  // namespace rbt
