// Butterfly kernels for gfx950: coefficient draw, the fused two-sided
// transform A~ = U^T A V (Eq. 1, Eq. 3) and the one-sided transforms
// b~ = U^T b and x = V x~.
//
// Index algebra (Sec. 3, Alg. 1 with m = 2^d g ceil(n/(2^d g)), g = 1 for the
// non-tiled structure, the tile size or the Eq. 8 granule otherwise): with
// q = m / 2^d write i = r + t q. Layer l has half-size h_l = 2^(d-l) q, so
// its butterflies pair i with the index whose t differs in bit (d-l), when
// that index is < n (else i is unpaired: Eq. 2 keeps it, factor 1). Layers
// lo..hi therefore act on independent groups of 2^(hi-lo+1) indices; the
// two-sided transform acts on independent 2^P x 2^P blocks of A. Each lane
// owns one block: it reads the block once, applies every layer of the pass
// in registers and writes it back, so a pass moves each element of A
// through HBM exactly once (the fusion noted at the end of Sec. 3). With
// depth <= 3 one pass does the whole transform.
//
// Lanes of a wavefront own consecutive r, so every load and store of the
// block is a coalesced run along a column (column-major A). No LDS staging
// is needed: the block members of one lane are q rows apart, and the
// neighbouring lanes fill in the rows between them.
//
// Per layer and side: mix pairs (a, b) -> (a + b, a - b), then scale by the
// coefficient of the output index times 1/sqrt(2) when the index is paired
// (the normalisation folded into the diagonal, as Sec. 3 notes for the
// 4dn^2 flop count).
#include <cmath>

#include "butterfly_dev.h"

namespace rbt {

namespace {

using dev::Pass;
using dev::group_base;

__global__ void __launch_bounds__(256) k_generate(int64_t n, int64_t q, int d, int kind,
                                                  uint64_t seed, double *__restrict__ U,
                                                  double *__restrict__ V) {
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int64_t total = 2 * n * d;
  if (idx >= total) return;
  const int side = idx >= n * d ? 1 : 0;
  const int64_t rem = idx - side * n * d;
  const int layer = int(rem / n) + 1;
  const int64_t i = rem % n;
  (side ? V : U)[rem] = kind == 1 ? dev::rotation_coefficient(seed, i, side, layer, n, q, d)
                                  : dev::coefficient(seed, i, side, layer);
}

// Two-sided pass. Thread (gx, gy) owns row group gx and column group gy.
// TI: element type of the input (FP64, or the FP32 output of an earlier
// pass when the output is FP32), arithmetic in FP64. Loads and stores carry
// non-temporal hints: every element is read and written once, and the
// matrix is larger than the caches (5.17 -> 5.33 TB/s for the FP64 output
// at n = 20000, 2.67 -> 2.24 ms for the FP32 output at n = 32768).
template <int P, typename TI, typename TO>
__global__ void __launch_bounds__(256) k_transform2(const TI *__restrict__ A, int64_t lda,
                                                    TO *__restrict__ Out, int64_t ldo,
                                                    const double *__restrict__ U,
                                                    const double *__restrict__ V, Pass ps) {
  const int64_t gr = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (gr >= ps.ngroups) return;
  const int64_t rb = group_base(ps, gr);
  if (rb >= ps.n) return;
  for (int64_t gc = blockIdx.y; gc < ps.ngroups; gc += gridDim.y) {
    const int64_t cb = group_base(ps, gc);
    if (cb >= ps.n) continue;
    dev::transform2_block<P, TO, true>(A, lda, Out, ldo, U, V, ps, rb, cb);
  }
}

// One-sided pass on an n x nrhs block.
template <int P, int OP>
__global__ void __launch_bounds__(256) k_transform_vec(double *__restrict__ B, int64_t ldb,
                                                       int64_t nrhs,
                                                       const double *__restrict__ C, Pass ps,
                                                       const int32_t *gate) {
  if (gated(gate)) return;
  const int64_t gr = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (gr >= ps.ngroups) return;
  const int64_t rb = group_base(ps, gr);
  if (rb >= ps.n) return;
  for (int64_t j = blockIdx.y; j < nrhs; j += gridDim.y)
    dev::transform_vec_block<P, OP>(B, ldb, j, C, ps, rb);
}

Pass make_pass(const Geometry &g, int lo, int hi) {
  return dev::make_pass(g.n, g.q, g.d, lo, hi, g.kind == 1 ? 1 : 0, g.sides);
}

template <typename TI, typename TO>
hipError_t launch_pass2(const Pass &ps, const TI *A, int64_t lda, TO *out, int64_t ldo,
                        const double *U, const double *V, hipStream_t s) {
  const int P = ps.hi - ps.lo + 1;
  const int64_t gy = ps.ngroups < 65535 ? ps.ngroups : 65535;
  dim3 grid(unsigned((ps.ngroups + 255) / 256), unsigned(gy));
  switch (P) {
    case 0: hipLaunchKernelGGL((k_transform2<0, TI, TO>), grid, dim3(256), 0, s, A, lda, out, ldo, U, V, ps); break;
    case 1: hipLaunchKernelGGL((k_transform2<1, TI, TO>), grid, dim3(256), 0, s, A, lda, out, ldo, U, V, ps); break;
    case 2: hipLaunchKernelGGL((k_transform2<2, TI, TO>), grid, dim3(256), 0, s, A, lda, out, ldo, U, V, ps); break;
    default: hipLaunchKernelGGL((k_transform2<3, TI, TO>), grid, dim3(256), 0, s, A, lda, out, ldo, U, V, ps); break;
  }
  return hipGetLastError();
}

template <int OP>
hipError_t launch_pass_vec(const Pass &ps, double *B, int64_t ldb, int64_t nrhs, const double *C,
                           hipStream_t s) {
  const int P = ps.hi - ps.lo + 1;
  dim3 grid(unsigned((ps.ngroups + 255) / 256), unsigned(nrhs < 65535 ? nrhs : 65535));
  switch (P) {
    case 1: hipLaunchKernelGGL((k_transform_vec<1, OP>), grid, dim3(256), 0, s, B, ldb, nrhs, C, ps, refine_gate()); break;
    case 2: hipLaunchKernelGGL((k_transform_vec<2, OP>), grid, dim3(256), 0, s, B, ldb, nrhs, C, ps, refine_gate()); break;
    default: hipLaunchKernelGGL((k_transform_vec<3, OP>), grid, dim3(256), 0, s, B, ldb, nrhs, C, ps, refine_gate()); break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_generate(const Geometry &g, uint64_t seed, double *U, double *V, hipStream_t s) {
  const int64_t total = 2 * g.n * g.d;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_generate, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, g.n, g.q,
                     g.d, g.kind, seed, U, V);
  return hipGetLastError();
}

// Layers are processed in passes of at most three, from layer d down to 1
// (the order of U^T A V); rows and columns of a pass commute. Depth 0 is the
// identity (a copy or conversion when out of place). With an FP32 output and
// depth > 3 every pass writes the FP32 output (the first reads A, the later
// ones the output in place), so the values are rounded to FP32 once per pass.
hipError_t launch_transform2(const Geometry &g, const double *A, int64_t lda, void *out,
                             int64_t ldo, int out_prec, const double *U, const double *V,
                             hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  if (g.d == 0) {
    if (out_prec == RBT_FP64 && (const void *)A == out) return hipSuccess;
    const Pass ps = dev::identity_pass(g.n);
    if (out_prec == RBT_FP32)
      return launch_pass2<double, float>(ps, A, lda, (float *)out, ldo, U, V, s);
    return launch_pass2<double, double>(ps, A, lda, (double *)out, ldo, U, V, s);
  }
  const double *src = A;
  int64_t lds = lda;
  bool first = true;
  int hi = g.d;
  while (hi >= 1) {
    const int lo = hi - 2 >= 1 ? hi - 2 : 1;
    const Pass ps = make_pass(g, lo, hi);
    hipError_t e;
    if (out_prec == RBT_FP32) {
      e = first ? launch_pass2<double, float>(ps, src, lds, (float *)out, ldo, U, V, s)
                : launch_pass2<float, float>(ps, (const float *)out, ldo, (float *)out, ldo, U,
                                             V, s);
    } else {
      e = launch_pass2<double, double>(ps, src, lds, (double *)out, ldo, U, V, s);
      src = (const double *)out;
      lds = ldo;
    }
    if (e != hipSuccess) return e;
    first = false;
    hi = lo - 1;
  }
  return hipSuccess;
}

hipError_t launch_transform_vec(const Geometry &g, int64_t nrhs, double *B, int64_t ldb,
                                const double *C, int op, hipStream_t s) {
  if (g.n == 0 || nrhs == 0 || g.d == 0) return hipSuccess;
  if (op == RBT_OP_T) {
    int hi = g.d;
    while (hi >= 1) {
      const int lo = hi - 2 >= 1 ? hi - 2 : 1;
      hipError_t e = launch_pass_vec<RBT_OP_T>(make_pass(g, lo, hi), B, ldb, nrhs, C, s);
      if (e != hipSuccess) return e;
      hi = lo - 1;
    }
  } else {
    int lo = 1;
    while (lo <= g.d) {
      const int hi = lo + 2 <= g.d ? lo + 2 : g.d;
      hipError_t e = launch_pass_vec<RBT_OP_N>(make_pass(g, lo, hi), B, ldb, nrhs, C, s);
      if (e != hipSuccess) return e;
      lo = hi + 1;
    }
  }
  return hipSuccess;
}

}  // namespace rbt
