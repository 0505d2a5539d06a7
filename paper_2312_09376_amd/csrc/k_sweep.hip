// Triangular sweeps for few right-hand sides (nrhs <= 16) as ONE persistent
// launch per sweep, for the solves after the elimination (Sec. 1, step 3:
// L y = b~, U x~ = y) and the adjoint solves.
//
// Each workgroup takes a ticket (atomic counter) and handles the block row
// of that rank in sweep order: it accumulates op(A)[b, j] x_j over the
// blocks j solved before it, then solves its diagonal block with the
// precomputed inverse (x = Di r; for FP64 factors and FP32 arithmetic one
// more step, x += Di (r - T x), keeps the backward error of substitution) and
// publishes x_b. The matrix entries of the next block are loaded before
// each wait, so the loads overlap it.
//
// Publication: every solution entry carries its own readiness. Before the
// sweep the launcher fills a publication buffer P (n x nrhs, in the sync
// area) with a signalling-NaN pattern that no arithmetic produces; a
// workgroup publishes x_b by storing its entries into P with agent-scope
// atomic stores (and into B, the output), and a workgroup that needs x_j
// polls its entries of P with agent-scope atomic loads until none holds the
// pattern. One 8-byte entry is written once per sweep and read whole, so a
// read value that is not the pattern is the published one: no fence, no
// counter and no second round trip sit between a block's solution and its
// consumers (the critical path of the sweep is one store and one load per
// block).
//
// Progress: a workgroup only waits for blocks of smaller tickets, which were
// taken by workgroups already running, so every wait ends. The spin is also
// bounded (spin_limit sleeps per entry, the library's option; a negative
// limit expires every wait at once, which tests use to reach this path): a
// workgroup whose wait expires uses NaN for that entry, sets the sticky
// error word sync[3] (which no sweep launch clears), stores NaN as its
// block's solution, so the result can never be a silently wrong finite
// vector, and goes on, so the grid always drains.
//
// Layout: 512 threads = 128 rows x 4 column segments of 32; products of a
// 128 x 128 block with the x block are reduced over the segments in LDS.
//
// Arithmetic type C: FP64 for FP64 factors. For the FP32 factors of the
// mixed-precision solve it is FP32: the right-hand side (FP64 storage, the
// transformed residual) is rounded to FP32 when loaded, the products, the
// diagonal-block inverses (FP32) and the reductions are FP32, and the FP32
// result is stored back widened; FP64 arithmetic with FP64 inverses is kept
// as an option.
#include <type_traits>

#include "internal.h"

namespace rbt {

namespace {

constexpr int TPB = 512;
constexpr int SEG = 4;
constexpr int SEGW = kNB / SEG;  // 32 columns per segment

template <TriMode MODE, typename TF>
__device__ __forceinline__ TF op_e(const TF *A, int64_t ld, int64_t m, int64_t k) {
  if constexpr (MODE == TriMode::LN || MODE == TriMode::UN)
    return A[m + k * ld];
  else
    return A[k + m * ld];
}

__device__ __forceinline__ double coherent_load(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void coherent_store(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Entry of P not yet published: a signalling NaN (arithmetic only yields
// quiet NaNs; a published entry with this pattern is stored as a quiet NaN).
constexpr uint64_t kUnpublished = 0x7FF4B1A5C0DE0001ull;
__device__ __forceinline__ bool unpublished(double v) {
  return __builtin_bit_cast(uint64_t, v) == kUnpublished;
}
// P: 256 bytes after the start of the sync area, column c at P + c n.
constexpr int kSyncPubOffsetInts = 64;

template <int NMAX, TriMode MODE, typename TF, bool REFINE, typename C>
__global__ void __launch_bounds__(TPB)
    k_sweep(int64_t n, int N, const TF *__restrict__ A, int64_t ld,
            const C *__restrict__ Winv, double *B, int64_t ldb, int32_t *sync, int64_t nb,
            int64_t spin_limit, const int32_t *gate) {
  // (the gate is read before any ticket is taken: every workgroup of a gated
  // launch returns here)
  if (gated(gate)) return;
  constexpr bool FWD = (MODE == TriMode::LN || MODE == TriMode::UT);
  constexpr bool UNIT = (MODE == TriMode::LN || MODE == TriMode::LT);
  __shared__ C xs[kNB][NMAX];
  __shared__ C part[SEG][kNB][NMAX];
  __shared__ int64_t tk;

  const int tid = threadIdx.x;
  const int i = tid & (kNB - 1), sg = tid >> 7;
  if (tid == 0) tk = atomicAdd(&sync[0], 1);
  __shared__ int expired_sh;
  if (tid == 0) expired_sh = 0;
  __syncthreads();
  const int64_t t = tk;
  if (t >= nb) return;
  int32_t *err = sync + 3;  // sticky: cleared by the entry points, not per sweep
  double *pub = reinterpret_cast<double *>(sync + kSyncPubOffsetInts);
  const int64_t b = FWD ? t : nb - 1 - t;
  const int64_t r0 = b * kNB;
  const int kb = int(n - r0 < kNB ? n - r0 : kNB);
  const int ir = i < kb ? i : kb - 1;  // clamped row for loads

  // sum over segments of part -> out (threads of segment 0)
  auto reduce = [&](const C (&a)[NMAX], C (&out)[NMAX]) {
#pragma unroll
    for (int c = 0; c < NMAX; ++c) part[sg][i][c] = a[c];
    __syncthreads();
    if (sg == 0) {
#pragma unroll
      for (int c = 0; c < NMAX; ++c)
        out[c] = (part[0][i][c] + part[1][i][c]) + (part[2][i][c] + part[3][i][c]);
    }
    __syncthreads();
  };

  // The diagonal block's inverse and the block's right-hand side do not
  // depend on other blocks: up to 8 right-hand sides they are loaded into
  // registers before any wait and leave the critical path of the sweep;
  // with 16 and FP32 factors the inverse is loaded right after the last
  // accumulation; with 16 and FP64 factors at each use.
  constexpr bool PRE = (NMAX <= 8);
  const C *Di = Winv + b * 2 * kNB * kNB +
                ((MODE == TriMode::LN || MODE == TriMode::LT) ? 0 : kNB * kNB);
  auto load_dinv = [&](C (&ev)[SEGW]) {
#pragma unroll
    for (int q = 0; q < SEGW; ++q) {
      const int jj = sg * SEGW + q;
      // Di is a full kNB x kNB allocation; entries beyond kb are masked
      const C v = (MODE == TriMode::LN || MODE == TriMode::UN) ? Di[i + jj * kNB]
                                                               : Di[jj + i * kNB];
      ev[q] = (i < kb && jj < kb) ? v : C(0);
    }
  };
  auto load_tdiag = [&](TF (&e)[SEGW]) {
#pragma unroll
    for (int q = 0; q < SEGW; ++q) {
      const int jj = sg * SEGW + q;
      e[q] = op_e<MODE>(A, ld, r0 + ir, r0 + (jj < kb ? jj : kb - 1));
    }
  };
  C dpre[PRE ? SEGW : 1];
  C bpre[PRE ? NMAX : 1];
  if constexpr (PRE) {
    load_dinv(dpre);
#pragma unroll
    for (int c = 0; c < NMAX; ++c)
      bpre[c] = (sg == 0 && i < kb && c < N) ? C(B[(r0 + i) + int64_t(c) * ldb]) : C(0);
  }

  // The diagonal block of the refinement step is loaded here too where
  // registers allow (one right-hand side; FP32 factors up to eight): after
  // the last wait its memory latency would sit on the sweep's critical path.
  constexpr bool PRE_T = REFINE && (NMAX == 1 || (sizeof(TF) == 4 && NMAX <= 8));
  TF etp[PRE_T ? SEGW : 1];
  if constexpr (PRE_T) load_tdiag(etp);

  // ---- accumulate op(A)[b, j] x_j over the blocks solved before b ----
  C acc[NMAX];
#pragma unroll
  for (int c = 0; c < NMAX; ++c) acc[c] = C(0);
  for (int64_t s = 0; s < t; ++s) {
    const int64_t j = FWD ? s : nb - 1 - s;
    const int64_t c0 = j * kNB;
    const int cb = int(n - c0 < kNB ? n - c0 : kNB);
    TF e[SEGW];
#pragma unroll
    for (int q = 0; q < SEGW; ++q) {
      const int col = sg * SEGW + q;
      e[q] = op_e<MODE>(A, ld, r0 + ir, c0 + (col < cb ? col : cb - 1));
    }
    // x_j from P, each entry polled until published (bounded). A thread's
    // entries (two or four with 8 or 16 right-hand sides) are all loaded
    // before any is waited on, so a published block costs one round trip.
    bool expired = false;
    constexpr int PER = (kNB * NMAX + TPB - 1) / TPB;
    // entry (k, c) sits at P[(c0 + k) + c n]: consecutive lanes take
    // consecutive k, so a wavefront's polls read contiguous memory
    if constexpr (PER == 1) {
      const int k = tid % kNB, c = tid / kNB;
      if (tid < kNB * NMAX) {
        C v = C(0);
        if (k < cb && c < N) {
          const double *p = pub + (c0 + k) + int64_t(c) * n;
          double xv = coherent_load(p);
          int64_t spins = 0;
          while (unpublished(xv)) {
            if (spins >= spin_limit) {  // expired: NaN for this entry, poison this block
              expired = true;
              xv = __builtin_nan("");
              break;
            }
            __builtin_amdgcn_s_sleep(1);
            ++spins;
            xv = coherent_load(p);
          }
          v = C(xv);
        }
        xs[k][c] = v;
      }
    } else {
      double xv[PER];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int idx = tid + q * TPB;
        const int k = idx % kNB, c = idx / kNB;
        xv[q] = 0.0;
        if (idx < kNB * NMAX && k < cb && c < N) xv[q] = coherent_load(pub + (c0 + k) + int64_t(c) * n);
      }
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int idx = tid + q * TPB;
        const int k = idx % kNB, c = idx / kNB;
        if (idx >= kNB * NMAX) continue;
        C v = C(0);
        if (k < cb && c < N) {
          const double *p = pub + (c0 + k) + int64_t(c) * n;
          int64_t spins = 0;
          while (unpublished(xv[q])) {
            if (spins >= spin_limit) {  // expired: NaN for this entry, poison this block
              expired = true;
              xv[q] = __builtin_nan("");
              break;
            }
            __builtin_amdgcn_s_sleep(1);
            ++spins;
            xv[q] = coherent_load(p);
          }
          v = C(xv[q]);
        }
        xs[k][c] = v;
      }
    }
    if (expired) {
      __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      expired_sh = 1;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < SEGW; ++q) {
      const int col = sg * SEGW + q;
      const C a = col < cb ? C(e[q]) : C(0);
#pragma unroll
      for (int c = 0; c < NMAX; ++c) acc[c] += a * xs[col][c];
    }
    __syncthreads();
  }

  // loads of the diagonal work, issued before the reductions (the FP64
  // diagonal block of the refinement step only while registers allow;
  // with one right-hand side it was loaded before the waits)
  constexpr bool EARLY_T = REFINE && NMAX <= 8;
  TF et[REFINE ? SEGW : 1];
  if constexpr (PRE_T) {
#pragma unroll
    for (int q = 0; q < SEGW; ++q) et[q] = etp[q];
  } else if constexpr (EARLY_T) {
    load_tdiag(et);
  }
  // 16 right-hand sides: FP32 factors take the inverse here; FP64 factors
  // (more registers live) load it at each use
  constexpr bool EARLY_D = !PRE && !REFINE;
  C dlate[EARLY_D ? SEGW : 1];
  if constexpr (EARLY_D) load_dinv(dlate);

  // ---- r = b_b - acc ----
  C r[NMAX];
  reduce(acc, r);
  if (sg == 0) {
#pragma unroll
    for (int c = 0; c < NMAX; ++c) {
      // rows beyond kb summed clamped loads: zero them
      C bv;
      if constexpr (PRE)
        bv = bpre[c];
      else
        bv = (i < kb && c < N) ? C(B[(r0 + i) + int64_t(c) * ldb]) : C(0);
      r[c] = (i < kb && c < N) ? bv - r[c] : C(0);
      xs[i][c] = r[c];
    }
  }
  __syncthreads();

  // product of the diagonal block's inverse with xs
  auto prod_dinv = [&](C (&out)[NMAX]) {
    C ev[SEGW];
    if constexpr (PRE) {
#pragma unroll
      for (int q = 0; q < SEGW; ++q) ev[q] = dpre[q];
    } else if constexpr (EARLY_D) {
#pragma unroll
      for (int q = 0; q < SEGW; ++q) ev[q] = dlate[q];
    } else {
      load_dinv(ev);
    }
    C a[NMAX];
#pragma unroll
    for (int c = 0; c < NMAX; ++c) a[c] = C(0);
#pragma unroll
    for (int q = 0; q < SEGW; ++q)
#pragma unroll
      for (int c = 0; c < NMAX; ++c) a[c] += ev[q] * xs[sg * SEGW + q][c];
    reduce(a, out);
  };

  // ---- x = Di r ----
  C x[NMAX];
  prod_dinv(x);
  if constexpr (REFINE) {
    // res = r - T x ; x += Di res
    if (sg == 0) {
#pragma unroll
      for (int c = 0; c < NMAX; ++c) xs[i][c] = x[c];
    }
    __syncthreads();
    if constexpr (!EARLY_T) load_tdiag(et);
    C a[NMAX];
#pragma unroll
    for (int c = 0; c < NMAX; ++c) a[c] = C(0);
#pragma unroll
    for (int q = 0; q < SEGW; ++q) {
      const int jj = sg * SEGW + q;
      C v = C(et[q]);
      if (jj >= kb || i >= kb) v = C(0);
      else if (jj == i) v = UNIT ? C(1) : v;
      else if (FWD ? (jj > i) : (jj < i)) v = C(0);
#pragma unroll
      for (int c = 0; c < NMAX; ++c) a[c] += v * xs[jj][c];
    }
    C tx[NMAX];
    reduce(a, tx);
    if (sg == 0) {
#pragma unroll
      for (int c = 0; c < NMAX; ++c) xs[i][c] = r[c] - tx[c];
    }
    __syncthreads();
    C dx[NMAX];
    prod_dinv(dx);
    if (sg == 0) {
#pragma unroll
      for (int c = 0; c < NMAX; ++c) x[c] += dx[c];
    }
  }

  // ---- publish x_b (NaN if a wait of this block expired): the output B
  // and the consumers' copy in P ----
  const bool poisoned = expired_sh != 0;
  if (sg == 0 && i < kb) {
#pragma unroll
    for (int c = 0; c < NMAX; ++c)
      if (c < N) {
        const double v = poisoned ? __builtin_nan("") : double(x[c]);
        B[(r0 + i) + int64_t(c) * ldb] = v;
        coherent_store(&pub[(r0 + i) + int64_t(c) * n], unpublished(v) ? __builtin_nan("") : v);
      }
  }
}

// Before a sweep: ticket and legacy words cleared, P (count entries) set to
// the unpublished pattern.
__global__ void k_sweep_reset(int32_t *sync, int64_t count) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g < 3) sync[g] = 0;
  double *pub = reinterpret_cast<double *>(sync + kSyncPubOffsetInts);
  const double u = __builtin_bit_cast(double, kUnpublished);
  for (int64_t k = g; k < count; k += int64_t(gridDim.x) * blockDim.x) pub[k] = u;
}

template <int NMAX, TriMode MODE, typename TF, typename C>
hipError_t sweep_t(int64_t n, int N, const TF *LU, int64_t ld, const C *Winv, double *B,
                   int64_t ldb, int32_t *sync, hipStream_t s) {
  // one refinement step per diagonal block for FP64 factors and for FP32
  // arithmetic (a product with an explicit FP32 inverse alone is accurate to
  // kappa(block) u32 only); FP64 arithmetic on FP32 factors needs none
  constexpr bool REFINE = std::is_same<TF, double>::value || std::is_same<C, float>::value;
  const int64_t nb = (n + kNB - 1) / kNB;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  // ticket and legacy words, and P for the N columns; the sticky error word
  // sync[3] is left alone
  const int64_t count = n * int64_t(N);
  const int64_t blocks = (count + 255) / 256 < 1024 ? (count + 255) / 256 : 1024;
  hipLaunchKernelGGL(k_sweep_reset, dim3(unsigned(blocks < 1 ? 1 : blocks)), dim3(256), 0, s, sync,
                     count);
  hipLaunchKernelGGL((k_sweep<NMAX, MODE, TF, REFINE, C>), dim3(unsigned(nb)), dim3(TPB), 0, s, n,
                     N, LU, ld, Winv, B, ldb, sync, nb, sweep_spin_limit(), refine_gate());
  return hipGetLastError();
}

template <int NMAX, typename TF, typename C>
hipError_t sweep_n(TriMode mode, int64_t n, int N, const TF *LU, int64_t ld, const C *Winv,
                   double *B, int64_t ldb, int32_t *sync, hipStream_t s) {
  switch (mode) {
    case TriMode::LN: return sweep_t<NMAX, TriMode::LN>(n, N, LU, ld, Winv, B, ldb, sync, s);
    case TriMode::UN: return sweep_t<NMAX, TriMode::UN>(n, N, LU, ld, Winv, B, ldb, sync, s);
    case TriMode::UT: return sweep_t<NMAX, TriMode::UT>(n, N, LU, ld, Winv, B, ldb, sync, s);
    default: return sweep_t<NMAX, TriMode::LT>(n, N, LU, ld, Winv, B, ldb, sync, s);
  }
}

template <typename TF, typename C>
hipError_t sweep_any(TriMode mode, int64_t n, int64_t nrhs, const TF *LU, int64_t ld,
                     const C *Winv, double *B, int64_t ldb, int32_t *sync, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  if (nrhs > kSkinnyMax || sync == nullptr) return hipErrorInvalidValue;
  const int N = int(nrhs);
  if (N <= 1) return sweep_n<1>(mode, n, N, LU, ld, Winv, B, ldb, sync, s);
  if (N <= 4) return sweep_n<4>(mode, n, N, LU, ld, Winv, B, ldb, sync, s);
  if (N <= 8) return sweep_n<8>(mode, n, N, LU, ld, Winv, B, ldb, sync, s);
  return sweep_n<16>(mode, n, N, LU, ld, Winv, B, ldb, sync, s);
}

}  // namespace

hipError_t launch_sweep(TriMode mode, int64_t n, int64_t nrhs, const double *LU, int64_t ld,
                        const double *Winv, double *B, int64_t ldb, int32_t *sync,
                        hipStream_t s) {
  return sweep_any(mode, n, nrhs, LU, ld, Winv, B, ldb, sync, s);
}
hipError_t launch_sweep(TriMode mode, int64_t n, int64_t nrhs, const float *LU, int64_t ld,
                        const double *Winv, double *B, int64_t ldb, int32_t *sync,
                        hipStream_t s) {
  return sweep_any(mode, n, nrhs, LU, ld, Winv, B, ldb, sync, s);
}
hipError_t launch_sweep(TriMode mode, int64_t n, int64_t nrhs, const float *LU, int64_t ld,
                        const float *Winv, double *B, int64_t ldb, int32_t *sync,
                        hipStream_t s) {
  return sweep_any(mode, n, nrhs, LU, ld, Winv, B, ldb, sync, s);
}

}  // namespace rbt
