// Diagonal-block kernel of the blocked elimination without pivoting.
//
// One workgroup of 512 threads factors a kb x kb diagonal block (kb <= 128)
// in place, A = L U with unit-lower L (Sec. 1, step 2: GENP). The block is
// held in LDS (column-major, leading dimension 129 so that row-wise and
// column-wise lane patterns are both bank-conflict free) and eliminated in
// eight 16-column steps:
//   1. the 16-column panel is factored right-looking, rank-1, by four of the
//      eight wavefronts, one row per lane; every wavefront keeps its own copy of
//      the panel's top 16 rows, so each pivot row is broadcast within the
//      wavefront with readlane and the 16 steps need no workgroup barrier;
//   2. the 16-row block of U to its right is solved by forward substitution
//      with the panel's unit-lower 16 x 16 block (four lanes per column);
//   3. the trailing block takes a rank-16 update on the FP64 matrix cores,
//      16 x 16 tiles shared out over the eight wavefronts (two per SIMD, so
//      one wavefront's LDS accesses overlap the other's products); each tile's
//      accumulator starts from the LDS values and the L operand is negated.
// Rows and columns beyond kb hold the identity, so they never disturb the
// active part. The arithmetic type C is FP64 for FP64 factors; for the FP32
// factors of the mixed-precision elimination it is FP32 (LDS, broadcasts,
// the FP32 matrix cores), or FP64 as an option, in which case the block is
// widened on load and rounded once on store. A zero pivot is recorded in
// *info (first one, 1-based, offset gofs) and the arithmetic continues with
// IEEE Inf/NaN.
#include "internal.h"
#include "mma16.h"

namespace rbt {

namespace {

constexpr int NB = kNB;  // 128
constexpr int LD = NB + 1;
constexpr int PW = 16;   // panel width
constexpr int NT = 512;  // threads
constexpr int NW = NT / 64;

template <typename T, typename C>
__global__ void __launch_bounds__(NT) k_diag_lu(int kb, T *__restrict__ A, int64_t lda,
                                                 int64_t gofs, int32_t *__restrict__ info) {
  typedef Mma16<C> M;
  typedef typename M::v4 c4;
  __shared__ C S[NB * LD];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lk = lane >> 4;

  // Staging: every load of a batch is issued before any is consumed, so the
  // batch costs one memory latency instead of one per element.
  {
    const int r = tid & (NB - 1), c0 = tid >> 7;  // row, first column (0..3)
    // unconditional loads at clamped valid indices, all 32 in flight,
    // masked afterwards
    T v[NB * NB / NT];
    const int rr = r < kb ? r : kb - 1;
#pragma unroll
    for (int i = 0; i < NB * NB / NT; ++i) {
      const int c = c0 + (NT / NB) * i;
      v[i] = A[rr + int64_t(c < kb ? c : kb - 1) * lda];
    }
#pragma unroll
    for (int i = 0; i < NB * NB / NT; ++i) {
      const int c = c0 + (NT / NB) * i;
      S[c * LD + r] = (r < kb && c < kb) ? C(v[i]) : ((r == c) ? C(1) : C(0));
    }
  }
  __syncthreads();

  for (int c0 = 0; c0 < kb; c0 += PW) {
    // ---- 1. panel factorization (rows >= c0, columns c0..c0+15) by all
    // four wavefronts: lanes 0..15 of every wavefront hold the panel's top
    // 16 rows and update their own copy (the copies see identical
    // operations), so each pivot row is broadcast within the wavefront with
    // readlane and no barrier is needed; lanes 16..63 hold one row below
    // them each (48 per wavefront). Rows above the pivot take a zero
    // multiplier. ----
    if (wave < 4) {
      const bool top = lane < PW;
      const int row = top ? c0 + lane : c0 + PW + wave * 48 + (lane - PW);
      const bool valid = row < NB;
      const int rr = valid ? row : NB - 1;
      C x[PW];
#pragma unroll
      for (int j = 0; j < PW; ++j) x[j] = S[(c0 + j) * LD + rr];
      // The loop body is kept free of branches (a zero pivot is found after
      // it; the reciprocal and the scaled entry are pinned before the
      // selects), so that the compiler can start a pivot's division while
      // the previous pivot's updates are still issuing.
#pragma unroll
      for (int cc = 0; cc < PW; ++cc) {
        C prow[PW];
#pragma unroll
        for (int j = cc; j < PW; ++j) prow[j] = wave_bcast(x[j], cc);
        const C p = prow[cc];
        const bool act = top ? lane > cc : valid;
        C rp = C(1) / p;  // one division per pivot (scaling as in LAPACK's getf2)
        __asm__ volatile("" : "+v"(rp));
        C lm = x[cc] * rp;
        __asm__ volatile("" : "+v"(lm));
        const C l = act ? lm : C(0);
        x[cc] = act ? l : x[cc];
#pragma unroll
        for (int j = cc + 1; j < PW; ++j) x[j] -= l * prow[j];
      }
      {  // first zero pivot of the panel: top lane j of wavefront 0 holds pivot j in x[j]
        C d = x[0];
#pragma unroll
        for (int j = 1; j < PW; ++j) d = lane == j ? x[j] : d;
        const unsigned long long z = __ballot(top && c0 + lane < kb && d == C(0));
        if (wave == 0 && lane == 0 && z != 0 && info != nullptr)
          atomicCAS(info, 0, int32_t(gofs + c0 + __ffsll(z)));
      }
      if ((top && wave == 0) || (!top && valid)) {
#pragma unroll
        for (int j = 0; j < PW; ++j) S[(c0 + j) * LD + row] = x[j];
      }
    }
    __syncthreads();

    const int c1 = c0 + PW;  // first column/row after the panel
    if (c1 >= NB) break;
    // ---- 2. U block row: rows c0..c0+15, columns c1..127, by forward
    // substitution with the unit-lower 16 x 16 block: four lanes per column
    // (lane q of a quad holds rows q, q + 4, q + 8, q + 12), column c1 + g
    // for quad g, the pivot entry passed on by a quad broadcast and the next
    // pivot's coefficients read during this one. Every entry sees the same
    // operations in the same order as one-lane-per-column substitution. ----
    {
      const int g = tid >> 2, q = tid & 3;
      const int colA = c1 + g;
      const bool hasA = colA < NB;
      const int ca = hasA ? colA : NB - 1;
      C ya[4];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) ya[jj] = S[ca * LD + c0 + q + 4 * jj];
      C tn[4];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) tn[jj] = S[c0 * LD + c0 + q + 4 * jj];
#pragma unroll
      for (int j = 0; j < PW; ++j) {  // pivot j: entries i > j lose L(i, j) y_j
        const int jc = j >> 2, qc = j & 3;
        C t[4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) t[jj] = tn[jj];
        if (j + 1 < PW) {
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) tn[jj] = S[(c0 + j + 1) * LD + c0 + q + 4 * jj];
        }
        __builtin_amdgcn_sched_barrier(0);
        const C ba = quad_bcast(ya[jc], qc);
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          if (4 * jj + 3 <= j) continue;
          const bool upd = 4 * jj > j || q + 4 * jj > j;
          const C na = fma_c(-t[jj], ba, ya[jj]);
          ya[jj] = upd ? na : ya[jj];
        }
      }
      if (hasA) {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) S[colA * LD + c0 + q + 4 * jj] = ya[jj];
      }
    }
    __syncthreads();
    // ---- 3. trailing rank-16 update on 16 x 16 tiles, two per wavefront
    // at a time (tiles t and t + NW), so their LDS loads overlap ----
    const int nt = (NB - c1) / PW;
    const int ntt = nt * nt;
    for (int t = wave; t < ntt; t += 2 * NW) {
      const bool two = t + NW < ntt;
      const int tb = two ? t + NW : t;
      const int i0 = c1 + PW * (t % nt), j0 = c1 + PW * (t / nt);
      const int i1 = c1 + PW * (tb % nt), j1 = c1 + PW * (tb / nt);
      c4 acc0, acc1;
      C a0[4], b0[4], a1[4], b1[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc0[v] = S[(j0 + l16) * LD + i0 + M::row(lk, v)];
        acc1[v] = S[(j1 + l16) * LD + i1 + M::row(lk, v)];
      }
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int k = c0 + 4 * kk + lk;
        a0[kk] = -S[k * LD + i0 + l16];
        b0[kk] = S[(j0 + l16) * LD + k];
        a1[kk] = -S[k * LD + i1 + l16];
        b1[kk] = S[(j1 + l16) * LD + k];
      }
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        acc0 = M::mma(a0[kk], b0[kk], acc0);
        acc1 = M::mma(a1[kk], b1[kk], acc1);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        S[(j0 + l16) * LD + i0 + M::row(lk, v)] = acc0[v];
        if (two) S[(j1 + l16) * LD + i1 + M::row(lk, v)] = acc1[v];
      }
    }
    __syncthreads();
  }

  {
    const int rr = tid & (NB - 1), c0 = tid >> 7;
#pragma unroll 16
    for (int i = 0; i < NB * NB / NT; ++i) {
      const int c = c0 + (NT / NB) * i;
      if (rr < kb && c < kb) A[rr + int64_t(c) * lda] = T(S[c * LD + rr]);
    }
  }
}

}  // namespace

template <typename T, typename C>
hipError_t diag_lu_t(int kb, T *A, int64_t lda, int64_t gofs, int32_t *info, hipStream_t s) {
  if (kb <= 0) return hipSuccess;
  if (kb > kNB) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_diag_lu<T, C>), dim3(1), dim3(NT), 0, s, kb, A, lda, gofs, info);
  return hipGetLastError();
}

hipError_t launch_diag_lu(int kb, double *A, int64_t lda, int64_t gofs, int32_t *info,
                          hipStream_t s) {
  return diag_lu_t<double, double>(kb, A, lda, gofs, info, s);
}
hipError_t launch_diag_lu(int kb, float *A, int64_t lda, int64_t gofs, int32_t *info,
                          bool fp64_arith, hipStream_t s) {
  return fp64_arith ? diag_lu_t<float, double>(kb, A, lda, gofs, info, s)
                    : diag_lu_t<float, float>(kb, A, lda, gofs, info, s);
}

}  // namespace rbt
