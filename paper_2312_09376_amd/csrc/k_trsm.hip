// Block triangular solves with a factored kb x kb diagonal block (kb <= 128)
// of the elimination, 16 rows (columns) at a time: the update from the
// blocks already solved runs on the FP64 matrix cores, and each 16 x 16
// diagonal block is solved by plain substitution, so the rounding behaviour
// is that of ordinary forward/back substitution except that a division by a
// pivot is a multiplication by its reciprocal (within one rounding of the
// quotient). (Multiplying by explicit inverses of the diagonal blocks, even
// 16 x 16 ones, raised the backward error several-fold on N(0,1) matrices
// with large growth.)
//
// The kernels are latency-bound chains of eight dependent steps, so every
// operand of the loop is staged in LDS once, with coalesced reads, before
// the first step: the 28 off-diagonal 16 x 16 blocks of the triangle in
// matrix-core operand order (56 KB), the eight diagonal blocks in the order
// the substitution reads them (16 KB), and each wavefront's right-hand-side
// strip (17 KB, padded rows). After that a wavefront only talks to its own
// strip, so the steps need no workgroup barrier (LDS accesses of one
// wavefront complete in issue order). 140 KB of LDS: one workgroup per CU.
//
// Substitution inside a diagonal block: the 64 lanes hold 16 independent
// right-hand sides x 4 lanes (a quad), lane q of a quad holding entries
// q, q + 4, q + 8, q + 12. At pivot j the owner lane scales its entry and
// a quad broadcast (DPP) hands it to the other three, which update their
// entries. Every entry sees the same operations in the same order as in
// one-lane-per-right-hand-side substitution.
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
// MFMA: 16 x 16 x 4 products in the arithmetic type C (mma16.h).
//
// The triangle (TT) and the right-hand sides (TB) may be stored in FP32
// (mixed-precision elimination). The arithmetic type C is FP64 for FP64
// factors; for FP32 factors it is FP32 (LDS, substitution and the FP32
// matrix cores), or FP64 as an option, in which case values are widened on
// load and rounded once on store.
#include "internal.h"
#include "mma16.h"

namespace rbt {

namespace {

constexpr int NB = kNB;  // 128
constexpr int IB = 16;
constexpr int NBK = NB / IB;  // 8 diagonal blocks
constexpr int BLK = IB * IB;  // 256 doubles per block
constexpr int NOFF = NBK * (NBK - 1) / 2;  // 28 off-diagonal blocks on one side
// A wavefront's strip holds 128 vectors of 16 doubles, 17 apart: with a
// stride of 16 (128 bytes) the lanes that each own one vector hit the same
// LDS banks when staging and storing it back (65 % of the LDS cycles were
// bank conflicts).
constexpr int SLD = IB + 1;

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

// Orders the LDS accesses of the lanes of one wavefront (no instruction).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// In-place substitution with one 16 x 16 diagonal block, quad layout: the
// calling lane holds x[jj] = entry q + 4 jj of its right-hand side; tq[j * 16
// + jj] is the coefficient of pivot j for entry q + 4 jj (reciprocal for
// j's own entry; zero where unused); pivots j >= bs are skipped. FWD: entries
// after the pivot are updated, else entries before it.
template <bool FWD, bool UNIT, typename C>
__device__ __forceinline__ void quad_substitute(C (&x)[4], const C *tq, int q, int bs) {
  C tn[4];
  const int j0 = FWD ? 0 : IB - 1;
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) tn[jj] = tq[j0 * IB + jj];
#pragma unroll
  for (int s = 0; s < IB; ++s) {
    const int j = FWD ? s : IB - 1 - s;
    const int jc = j >> 2, qc = j & 3;
    C t[4];
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) t[jj] = tn[jj];
    if (s + 1 < IB) {  // next pivot's coefficients in flight during this one
      const int jn = FWD ? j + 1 : j - 1;
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) tn[jj] = tq[jn * IB + jj];
    }
    __builtin_amdgcn_sched_barrier(0);
    if (j < bs) {
      if constexpr (!UNIT) {
        const C xs = x[jc] * t[jc];
        x[jc] = q == qc ? xs : x[jc];
      }
      const C b = quad_bcast(x[jc], qc);
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        if (FWD ? (4 * jj + 3 <= j) : (4 * jj >= j)) continue;  // no entry of jj on that side
        const C nx = fma_c(-t[jj], b, x[jj]);
        const bool all = FWD ? (4 * jj > j) : (4 * jj + 3 < j);
        x[jj] = (all || (FWD ? q + 4 * jj > j : q + 4 * jj < j)) ? nx : x[jj];
      }
    }
  }
}

// BATCH: blockIdx.y selects diagonal block b of an n x n factor (T and B
// offset by b * kNB (1 + ldt) and b * bstride, kb = min(kNB, n - b kNB)), and
// the right-hand side is the identity (X = op(T_bb)^-1): used to form the
// inverses of the diagonal blocks once per factorization.
// LDS of one workgroup of either solve: diagonal blocks, off-diagonal
// blocks, four right-hand-side strips (136 KB).
template <typename C>
struct TrsmSmem {
  __attribute__((aligned(16))) C dblk[NBK * BLK];
  __attribute__((aligned(16))) C oblk[NOFF * BLK];
  __attribute__((aligned(16))) C strip[4][NB * SLD];
};

// Left solve of the 64 columns [64 bx, 64 bx + 64) of B.
template <TriMode MODE, bool BATCH, typename TT, typename TB, typename C>
__device__ __forceinline__ void trsm_left_body(int kb, int64_t N, const TT *T, int64_t ldt,
                                               TB *B, int64_t ldb, int64_t n, int64_t bstride,
                                               int64_t bx, TrsmSmem<C> &sm) {
  typedef Mma16<C> M;
  typedef typename M::v4 c4;
  typedef C c2 __attribute__((ext_vector_type(2)));
  if constexpr (BATCH) {
    const int64_t b = blockIdx.y;
    const int64_t r0 = b * NB;
    kb = int(n - r0 < NB ? n - r0 : NB);
    N = kb;
    T += r0 + r0 * ldt;
    B += b * bstride;
  }
  // dblk: op(T)(i, j) of diagonal block b at b*256 + j*16 + (i%4)*4 + i/4
  // (reciprocal on the diagonal of non-unit modes); ablk: off-diagonal block
  // (I, J), J before I, at p*256 + lane*4 + kk = op(T)(16I + l16, 16J + 4kk +
  // lk), p = I(I-1)/2 + J (forward) or J(J-1)/2 + I (backward)
  C *dblk = sm.dblk;
  C *ablk = sm.oblk;
  constexpr bool FWD = forward_order<MODE>();
  constexpr bool TRANS = MODE == TriMode::UT || MODE == TriMode::LT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  C *strip = sm.strip[wave];  // row-major 128 x 16
  const int64_t col0 = bx * 64 + wave * 16;

  {  // stage the diagonal blocks and the off-diagonal operands, coalesced:
     // consecutive threads read consecutive addresses of the stored T
    const int f = threadIdx.x & 15, g = threadIdx.x >> 4;
    const int i = TRANS ? g : f, j = TRANS ? f : g;  // element (i, j) of a block of op(T)
    TT raw[NBK];
#pragma unroll
    for (int b = 0; b < NBK; ++b)
      raw[b] = op_t<MODE>(T, ldt, clampi(IB * b + i, kb - 1), clampi(IB * b + j, kb - 1));
#pragma unroll
    for (int b = 0; b < NBK; ++b) {
      const int gi = IB * b + i, gj = IB * b + j;
      C v = (gi < kb && gj < kb) ? C(raw[b]) : (i == j ? C(1) : C(0));
      if (!unit_diag<MODE>() && i == j) v = C(1) / v;
      dblk[b * BLK + j * IB + (i & 3) * 4 + (i >> 2)] = v;
    }
    TT oraw[NOFF];
#pragma unroll
    for (int p = 0, I = 1; I < NBK; ++I)
#pragma unroll
      for (int J = 0; J < I; ++J, ++p) {
        // forward: block (I, J) below the diagonal; backward: (J, I) above it
        const int bi = FWD ? I : J, bj = FWD ? J : I;
        oraw[p] = op_t<MODE>(T, ldt, clampi(IB * bi + i, kb - 1), clampi(IB * bj + j, kb - 1));
      }
    const int slot = (16 * (j & 3) + i) * 4 + (j >> 2);  // lane (lk = j%4, l16 = i), kk = j/4
#pragma unroll
    for (int p = 0, I = 1; I < NBK; ++I)
#pragma unroll
      for (int J = 0; J < I; ++J, ++p) {
        const int bi = FWD ? I : J, bj = FWD ? J : I;
        const int gi = IB * bi + i, gj = IB * bj + j;
        ablk[p * BLK + slot] = (gi < kb && gj < kb) ? C(oraw[p]) : C(0);
      }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {  // strip: lane = row (two halves), 16 columns
    const int row = lane + 64 * h;
    if constexpr (BATCH) {
#pragma unroll
      for (int c = 0; c < IB; ++c) {
        const int64_t col = col0 + c;
        strip[row * SLD + c] = (row < kb && col < N && row == col) ? C(1) : C(0);
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
        strip[row * SLD + c] = (row < kb && col0 + c < N) ? C(raw[c]) : C(0);
    }
  }
  __syncthreads();

  const int nbk = (kb + IB - 1) / IB;
  const int cc = lane >> 2, q = lane & 3;  // substitution: right-hand side cc, entries q + 4 jj
  for (int step = 0; step < nbk; ++step) {
    const int I = FWD ? step : nbk - 1 - step;
    c4 acc0 = {C(0), C(0), C(0), C(0)}, acc1 = {C(0), C(0), C(0), C(0)};
#pragma unroll
    for (int s2 = 0; s2 < NBK - 1; ++s2) {
      if (s2 < step) {
        const int J = FWD ? s2 : nbk - 1 - s2;
        const int p = FWD ? I * (I - 1) / 2 + J : J * (J - 1) / 2 + I;
        const c2 a01 = *reinterpret_cast<const c2 *>(ablk + p * BLK + lane * 4);
        const c2 a23 = *reinterpret_cast<const c2 *>(ablk + p * BLK + lane * 4 + 2);
        const int k0 = IB * J + lk;
        acc0 = M::mma(a01[0], strip[(k0) * SLD + l16], acc0);
        acc1 = M::mma(a01[1], strip[(k0 + 4) * SLD + l16], acc1);
        acc0 = M::mma(a23[0], strip[(k0 + 8) * SLD + l16], acc0);
        acc1 = M::mma(a23[1], strip[(k0 + 12) * SLD + l16], acc1);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) strip[(IB * I + M::row(lk, v)) * SLD + l16] -= acc0[v] + acc1[v];
    wave_sync();
    const int bs = kb - IB * I < IB ? kb - IB * I : IB;
    const int o = IB * I;
    C x[4];
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) x[jj] = strip[(o + q + 4 * jj) * SLD + cc];
    quad_substitute<FWD, unit_diag<MODE>()>(x, dblk + I * BLK + q * 4, q, bs);
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
      strip[(o + q + 4 * jj) * SLD + cc] = (q + 4 * jj < bs) ? x[jj] : C(0);
    wave_sync();
  }

#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int row = lane + 64 * h;
#pragma unroll
    for (int c = 0; c < IB; ++c) {
      const int64_t col = col0 + c;
      if (row < kb && col < N) B[row + col * ldb] = TB(strip[row * SLD + c]);
    }
  }
}

template <TriMode MODE, bool BATCH, typename TT, typename TB, typename C>
__global__ void __launch_bounds__(256, 1) k_trsm_left(int kb, int64_t N, const TT *T,
                                                      int64_t ldt, TB *B, int64_t ldb,
                                                      int64_t n, int64_t bstride) {
  __shared__ TrsmSmem<C> sm;
  trsm_left_body<MODE, BATCH, TT, TB, C>(kb, N, T, ldt, B, ldb, n, bstride,
                                         int64_t(blockIdx.x), sm);
}

// Right solve of the 64 rows [64 bx, 64 bx + 64) of B.
template <typename TT, typename C>
__device__ __forceinline__ void trsm_right_upper_body(int kb, int64_t M, const TT *T, int64_t ldt,
                                                      TT *B, int64_t ldb, int64_t bx,
                                                      TrsmSmem<C> &sm) {
  typedef Mma16<C> Mm;
  typedef typename Mm::v4 c4;
  typedef C c2 __attribute__((ext_vector_type(2)));
  // dblk: U(r, c) of diagonal block b at b*256 + r*16 + (c%4)*4 + c/4
  // (reciprocal on the diagonal); ublk: block (I, J), I < J, at p*256 +
  // lane*4 + kk = U(16I + 4kk + lk, 16J + l16), p = J(J-1)/2 + I
  C *dblk = sm.dblk;
  C *ublk = sm.oblk;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  C *strip = sm.strip[wave];  // column-major 16 x 128
  const int64_t row0 = bx * 64 + wave * 16;

  {  // stage the triangle, consecutive threads on consecutive rows of U
    const int r = threadIdx.x % IB, c = threadIdx.x / IB;
    TT raw[NBK];
#pragma unroll
    for (int b = 0; b < NBK; ++b)
      raw[b] = T[clampi(IB * b + r, kb - 1) + int64_t(clampi(IB * b + c, kb - 1)) * ldt];
#pragma unroll
    for (int b = 0; b < NBK; ++b) {
      const int gi = IB * b + r, gj = IB * b + c;
      C v = (gi < kb && gj < kb) ? C(raw[b]) : (r == c ? C(1) : C(0));
      if (r == c) v = C(1) / v;
      dblk[b * BLK + r * IB + (c & 3) * 4 + (c >> 2)] = v;
    }
    TT uraw[NOFF];
#pragma unroll
    for (int p = 0, J = 1; J < NBK; ++J)
#pragma unroll
      for (int I = 0; I < J; ++I, ++p)
        uraw[p] = T[clampi(IB * I + r, kb - 1) + int64_t(clampi(IB * J + c, kb - 1)) * ldt];
    const int slot = (16 * (r & 3) + c) * 4 + (r >> 2);  // lane (lk = r%4, l16 = c), kk = r/4
#pragma unroll
    for (int p = 0, J = 1; J < NBK; ++J)
#pragma unroll
      for (int I = 0; I < J; ++I, ++p) {
        const int gi = IB * I + r, gj = IB * J + c;
        ublk[p * BLK + slot] = (gi < kb && gj < kb) ? C(uraw[p]) : C(0);
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
        strip[c * SLD + r] = (row < M && c < kb) ? C(raw[u]) : C(0);
      }
    }
  }
  __syncthreads();

  const int nbk = (kb + IB - 1) / IB;
  const int rq = lane >> 2, q = lane & 3;  // substitution: row rq, entries q + 4 jj
  for (int J = 0; J < nbk; ++J) {
    c4 acc0 = {C(0), C(0), C(0), C(0)}, acc1 = {C(0), C(0), C(0), C(0)};
#pragma unroll
    for (int I = 0; I < NBK - 1; ++I) {
      if (I < J) {
        const int p = J * (J - 1) / 2 + I;
        const c2 b01 = *reinterpret_cast<const c2 *>(ublk + p * BLK + lane * 4);
        const c2 b23 = *reinterpret_cast<const c2 *>(ublk + p * BLK + lane * 4 + 2);
        const int k0 = IB * I + lk;
        acc0 = Mm::mma(strip[(k0) * SLD + l16], b01[0], acc0);
        acc1 = Mm::mma(strip[(k0 + 4) * SLD + l16], b01[1], acc1);
        acc0 = Mm::mma(strip[(k0 + 8) * SLD + l16], b23[0], acc0);
        acc1 = Mm::mma(strip[(k0 + 12) * SLD + l16], b23[1], acc1);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) strip[(IB * J + l16) * SLD + Mm::row(lk, v)] -= acc0[v] + acc1[v];
    wave_sync();
    const int bs = kb - IB * J < IB ? kb - IB * J : IB;
    const int o = IB * J;
    C x[4];
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) x[jj] = strip[(o + q + 4 * jj) * SLD + rq];
    quad_substitute<true, false>(x, dblk + J * BLK + q * 4, q, bs);
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
      strip[(o + q + 4 * jj) * SLD + rq] = (q + 4 * jj < bs) ? x[jj] : C(0);
    wave_sync();
  }

  {
    const int r = lane % IB, cg = lane / IB;
    const int64_t row = row0 + r;
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const int c = cg + 4 * u;
      if (row < M && c < kb) B[row + int64_t(c) * ldb] = TT(strip[c * SLD + r]);
    }
  }
}

template <typename TT, typename C>
__global__ void __launch_bounds__(256, 1) k_trsm_right_upper(int kb, int64_t M, const TT *T,
                                                             int64_t ldt, TT *B, int64_t ldb) {
  __shared__ TrsmSmem<C> sm;
  trsm_right_upper_body<TT, C>(kb, M, T, ldt, B, ldb, int64_t(blockIdx.x), sm);
}

// Both solves of a panel step with one factored diagonal block, which are
// independent: L21 = A21 U11^-1 (the first gr workgroups, 64 rows each) and
// U12 = L11^-1 A12 for the panel's columns to the right (the rest, 64
// columns each). One launch instead of two, and the short left solve runs
// beside the right one.
template <typename TT, typename C>
__global__ void __launch_bounds__(256, 1) k_panel_trsm(int kb, int64_t M, int64_t N, const TT *T,
                                                       int64_t ldt, TT *Br, TT *Bl, int64_t ldb,
                                                       int64_t gr) {
  __shared__ TrsmSmem<C> sm;
  const int64_t bx = blockIdx.x;
  if (bx < gr)
    trsm_right_upper_body<TT, C>(kb, M, T, ldt, Br, ldb, bx, sm);
  else
    trsm_left_body<TriMode::LN, false, TT, TT, C>(kb, N, T, ldt, Bl, ldb, int64_t(0),
                                                  int64_t(0), bx - gr, sm);
}

template <typename TT, typename TB, typename C>
hipError_t trsm_left_t(TriMode mode, int kb, int64_t N, const TT *T, int64_t ldt, TB *B,
                       int64_t ldb, hipStream_t s) {
  if (kb <= 0 || N <= 0) return hipSuccess;
  if (kb > kNB) return hipErrorInvalidValue;
  const dim3 grid(unsigned((N + 63) / 64));
  const int64_t z = 0;
  switch (mode) {
    case TriMode::LN: hipLaunchKernelGGL((k_trsm_left<TriMode::LN, false, TT, TB, C>), grid, dim3(256), 0, s, kb, N, T, ldt, B, ldb, z, z); break;
    case TriMode::UN: hipLaunchKernelGGL((k_trsm_left<TriMode::UN, false, TT, TB, C>), grid, dim3(256), 0, s, kb, N, T, ldt, B, ldb, z, z); break;
    case TriMode::UT: hipLaunchKernelGGL((k_trsm_left<TriMode::UT, false, TT, TB, C>), grid, dim3(256), 0, s, kb, N, T, ldt, B, ldb, z, z); break;
    case TriMode::LT: hipLaunchKernelGGL((k_trsm_left<TriMode::LT, false, TT, TB, C>), grid, dim3(256), 0, s, kb, N, T, ldt, B, ldb, z, z); break;
  }
  return hipGetLastError();
}

// Inverses of the diagonal blocks, in the arithmetic and storage type C of W.
template <typename TT, typename C>
hipError_t diag_inverses_t(int64_t n, const TT *LU, int64_t ld, C *W, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + NB - 1) / NB;
  if (nb > 65535) return hipErrorInvalidValue;
  const dim3 grid(2, unsigned(nb));  // 2 x 64 columns of each 128 x 128 block
  // L^-1 at W + b * 2 kNB^2, U^-1 at W + b * 2 kNB^2 + kNB^2, each ld kNB
  hipLaunchKernelGGL((k_trsm_left<TriMode::LN, true, TT, C, C>), grid, dim3(256), 0, s, NB,
                     int64_t(NB), LU, ld, W, int64_t(NB), n, int64_t(2 * NB * NB));
  hipLaunchKernelGGL((k_trsm_left<TriMode::UN, true, TT, C, C>), grid, dim3(256), 0, s, NB,
                     int64_t(NB), LU, ld, W + NB * NB, int64_t(NB), n, int64_t(2 * NB * NB));
  return hipGetLastError();
}

template <typename TT, typename C>
hipError_t panel_trsm_t(int kb, int64_t M, int64_t N, const TT *T, int64_t ldt, TT *Br, TT *Bl,
                        int64_t ldb, hipStream_t s) {
  if (kb <= 0 || (M <= 0 && N <= 0)) return hipSuccess;
  if (kb > kNB) return hipErrorInvalidValue;
  const int64_t gr = M > 0 ? (M + 63) / 64 : 0, gl = N > 0 ? (N + 63) / 64 : 0;
  if (gr + gl > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_panel_trsm<TT, C>), dim3(unsigned(gr + gl)), dim3(256), 0, s, kb, M, N, T,
                     ldt, Br, Bl, ldb, gr);
  return hipGetLastError();
}

template <typename TT, typename C>
hipError_t trsm_right_upper_t(int kb, int64_t M, const TT *T, int64_t ldt, TT *B, int64_t ldb,
                              hipStream_t s) {
  if (kb <= 0 || M <= 0) return hipSuccess;
  if (kb > kNB) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_trsm_right_upper<TT, C>), dim3(unsigned((M + 63) / 64)), dim3(256), 0, s,
                     kb, M, T, ldt, B, ldb);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_trsm_left(TriMode mode, int kb, int64_t N, const double *T, int64_t ldt,
                            double *B, int64_t ldb, hipStream_t s) {
  return trsm_left_t<double, double, double>(mode, kb, N, T, ldt, B, ldb, s);
}
hipError_t launch_trsm_left(TriMode mode, int kb, int64_t N, const float *T, int64_t ldt, float *B,
                            int64_t ldb, bool fp64_arith, hipStream_t s) {
  return fp64_arith ? trsm_left_t<float, float, double>(mode, kb, N, T, ldt, B, ldb, s)
                    : trsm_left_t<float, float, float>(mode, kb, N, T, ldt, B, ldb, s);
}
hipError_t launch_diag_inverses(int64_t n, const double *LU, int64_t ld, double *W,
                                hipStream_t s) {
  return diag_inverses_t(n, LU, ld, W, s);
}
hipError_t launch_diag_inverses(int64_t n, const float *LU, int64_t ld, double *W, hipStream_t s) {
  return diag_inverses_t(n, LU, ld, W, s);
}
hipError_t launch_diag_inverses(int64_t n, const float *LU, int64_t ld, float *W, hipStream_t s) {
  return diag_inverses_t(n, LU, ld, W, s);
}
hipError_t launch_trsm_right_upper(int kb, int64_t M, const double *T, int64_t ldt, double *B,
                                   int64_t ldb, hipStream_t s) {
  return trsm_right_upper_t<double, double>(kb, M, T, ldt, B, ldb, s);
}
hipError_t launch_trsm_right_upper(int kb, int64_t M, const float *T, int64_t ldt, float *B,
                                   int64_t ldb, bool fp64_arith, hipStream_t s) {
  return fp64_arith ? trsm_right_upper_t<float, double>(kb, M, T, ldt, B, ldb, s)
                    : trsm_right_upper_t<float, float>(kb, M, T, ldt, B, ldb, s);
}
hipError_t launch_panel_trsm(int kb, int64_t M, int64_t N, const double *T, int64_t ldt,
                             double *Br, double *Bl, int64_t ldb, hipStream_t s) {
  return panel_trsm_t<double, double>(kb, M, N, T, ldt, Br, Bl, ldb, s);
}
hipError_t launch_panel_trsm(int kb, int64_t M, int64_t N, const float *T, int64_t ldt, float *Br,
                             float *Bl, int64_t ldb, bool fp64_arith, hipStream_t s) {
  return fp64_arith ? panel_trsm_t<float, double>(kb, M, N, T, ldt, Br, Bl, ldb, s)
                    : panel_trsm_t<float, float>(kb, M, N, T, ldt, Br, Bl, ldb, s);
}

}  // namespace rbt
