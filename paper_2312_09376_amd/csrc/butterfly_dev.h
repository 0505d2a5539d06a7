// Device-side butterfly building blocks shared by the grid kernels
// (k_butterfly.hip) and the batched persistent kernel (k_batched.hip).
//
// Index algebra (Sec. 3, Alg. 1 with non-tiled m = 2^d ceil(n/2^d)): with
// q = m / 2^d write i = r + t q. Layer l has half-size h_l = 2^(d-l) q, so
// its butterflies pair i with the index whose t differs in bit (d-l), when
// that index is < n (else i is unpaired: Eq. 2 keeps it, factor 1). Layers
// lo..hi therefore act on independent groups of 2^(hi-lo+1) indices.
//
// Per layer and side: mix pairs (a, b) -> (a + b, a - b), then scale by the
// coefficient of the output index times 1/sqrt(2) when the index is paired
// (the normalisation folded into the diagonal, as Sec. 3 notes for the
// 4dn^2 flop count).
//
// Rotation butterflies (Sec. 3, the block-rotation form with R_l = I): a pair
// (a, b) becomes (c x_a + s x_b, s x_a - c x_b) with c, s the packed
// coefficients at a and b (cos and sin of the pair's angle); unpaired indices
// are left as they are (a rotation by 0 degrees). Each layer is symmetric, so
// U^T and U differ only in the order of the layers.
// One-sided RBT (Sec. 7): only the rows are transformed (A~ = U^T A).
#ifndef RBT_BUTTERFLY_DEV_H
#define RBT_BUTTERFLY_DEV_H

#include "internal.h"

namespace rbt {
namespace dev {

constexpr double kInvSqrt2 = 0.70710678118654752440;

// SplitMix64 output number c (0-based) of the generator started at `seed`
// (Steele, Lea, Flood 2014), in counter form.
__device__ __forceinline__ uint64_t splitmix_at(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Coefficient of index i, side (0 = U, 1 = V), layer (1-based): exp(r/20),
// r = 2 u - 1 with u the top 53 bits of draw 128 i + 64 side + layer - 1.
__device__ __forceinline__ double coefficient(uint64_t seed, int64_t i, int side, int layer) {
  const uint64_t c = 128ull * uint64_t(i) + 64ull * uint64_t(side) + uint64_t(layer - 1);
  const double u = double(splitmix_at(seed, c) >> 11) * 0x1.0p-53;
  return exp((2.0 * u - 1.0) / 20.0);
}

// Geometry of one pass over layers lo..hi (P = hi - lo + 1 <= 3), and the
// butterfly kind (rot: rotation butterflies) and sides (2, or 1 for the
// one-sided transform of the rows only).
struct Pass {
  int64_t n, q;
  int d, lo, hi;
  int64_t stride;   // 2^(d-hi) q : partner distance of layer hi
  int64_t ngroups;  // m / 2^P
  int rot, sides;
};

__host__ __device__ inline Pass make_pass(int64_t n, int64_t q, int d, int lo, int hi,
                                          int rot = 0, int sides = 2) {
  Pass ps;
  ps.n = n;
  ps.q = q;
  ps.d = d;
  ps.lo = lo;
  ps.hi = hi;
  ps.stride = q << (d - hi);
  ps.ngroups = (q << d) >> (hi - lo + 1);
  ps.rot = rot;
  ps.sides = sides;
  return ps;
}

// Depth 0: every index is its own group (identity; copy or conversion).
__host__ __device__ inline Pass identity_pass(int64_t n) {
  Pass ps;
  ps.n = n; ps.q = n; ps.d = 0; ps.lo = 1; ps.hi = 0; ps.stride = n; ps.ngroups = n;
  ps.rot = 0; ps.sides = 2;
  return ps;
}

// Packed rotation coefficient of index i in layer `layer` for the structure
// (n, q, d): cos(theta) at the top index of a pair, sin(theta) at the bottom
// one, 1 for an unpaired index; theta = 2 pi u, u the uniform of the
// coefficient counter at the pair's top index.
__device__ __forceinline__ double rotation_coefficient(uint64_t seed, int64_t i, int side,
                                                       int layer, int64_t n, int64_t q, int d) {
  const int64_t r = i % q, t = i / q;
  const int64_t bit = int64_t(1) << (d - layer);
  const int64_t j = r + (t ^ bit) * q;
  if (j >= n) return 1.0;
  const bool top = (t & bit) == 0;
  const int64_t a = top ? i : j;
  const uint64_t c = 128ull * uint64_t(a) + 64ull * uint64_t(side) + uint64_t(layer - 1);
  const double u = double(splitmix_at(seed, c) >> 11) * 0x1.0p-53;
  const double th = 2.0 * 3.14159265358979323846 * u;
  return top ? cos(th) : sin(th);
}

// First index of group g.
__device__ __forceinline__ int64_t group_base(const Pass &ps, int64_t g) {
  const int64_t r = g % ps.q;
  const int64_t rest = g / ps.q;
  const int lowbits = ps.d - ps.hi;
  const int64_t tl = rest & ((int64_t(1) << lowbits) - 1);
  const int64_t th = rest >> lowbits;
  return r + ps.q * (tl + (th << (ps.d - ps.lo + 1)));
}

template <typename T>
__device__ __forceinline__ T convert_out(double x);
template <>
__device__ __forceinline__ double convert_out<double>(double x) { return x; }
template <>
__device__ __forceinline__ float convert_out<float>(double x) { return float(x); }

// Two-sided pass on the block (row group at rb) x (column group at cb):
// read once, all layers of the pass in registers, write once.
// (Pointer types are template parameters so that callers can pass pointers
// qualified with the global address space.)
// STREAM: A is read and the output written with non-temporal hints (data
// touched once, larger than the caches); callers that read the output back
// soon (the batched kernel) keep the default.
template <int P, typename TO, bool STREAM = false, typename PA, typename PO, typename PC>
__device__ __forceinline__ void transform2_block(PA __restrict__ A, int64_t lda,
                                                 PO __restrict__ Out, int64_t ldo,
                                                 PC __restrict__ U, PC __restrict__ V,
                                                 const Pass &ps, int64_t rb, int64_t cb) {
  constexpr int G = 1 << P;
  int64_t ri[G], ci[G];
  bool rv[G], cv[G];
#pragma unroll
  for (int p = 0; p < G; ++p) {
    ri[p] = rb + p * ps.stride;
    rv[p] = ri[p] < ps.n;
    ci[p] = cb + p * ps.stride;
    cv[p] = ci[p] < ps.n;
  }
  double x[G][G];
#pragma unroll
  for (int c = 0; c < G; ++c)
#pragma unroll
    for (int r = 0; r < G; ++r) {
      if constexpr (STREAM)
        x[r][c] = (rv[r] && cv[c]) ? __builtin_nontemporal_load(&A[ri[r] + ci[c] * lda]) : 0.0;
      else
        x[r][c] = (rv[r] && cv[c]) ? A[ri[r] + ci[c] * lda] : 0.0;
    }
  const bool two = ps.sides != 1;
#pragma unroll
  for (int bit = 0; bit < P; ++bit) {
    // layer l = hi - bit pairs block members p and p ^ (1 << bit)
    const int l = ps.hi - bit;
    const int64_t off = int64_t(l - 1) * ps.n;
    if (ps.rot) {
#pragma unroll
      for (int p = 0; p < G; ++p) {  // rows
        if (p & (1 << bit)) continue;
        const int p2 = p | (1 << bit);
        if (!rv[p2]) continue;
        const double c = U[off + ri[p]], sn = U[off + ri[p2]];
#pragma unroll
        for (int cc = 0; cc < G; ++cc) {
          const double a = x[p][cc], b = x[p2][cc];
          x[p][cc] = c * a + sn * b;
          x[p2][cc] = sn * a - c * b;
        }
      }
      if (two) {
#pragma unroll
        for (int p = 0; p < G; ++p) {  // columns
          if (p & (1 << bit)) continue;
          const int p2 = p | (1 << bit);
          if (!cv[p2]) continue;
          const double c = V[off + ci[p]], sn = V[off + ci[p2]];
#pragma unroll
          for (int r = 0; r < G; ++r) {
            const double a = x[r][p], b = x[r][p2];
            x[r][p] = c * a + sn * b;
            x[r][p2] = sn * a - c * b;
          }
        }
      }
      continue;
    }
    double fr[G], fc[G];
#pragma unroll
    for (int p = 0; p < G; ++p) {
      const int p2 = p ^ (1 << bit);
      const double sr = (rv[p] && rv[p2]) ? kInvSqrt2 : 1.0;
      const double sc = (cv[p] && cv[p2]) ? kInvSqrt2 : 1.0;
      fr[p] = rv[p] ? U[off + ri[p]] * sr : 0.0;
      fc[p] = two ? (cv[p] ? V[off + ci[p]] * sc : 0.0) : 1.0;
    }
#pragma unroll
    for (int p = 0; p < G; ++p) {  // rows
      if (p & (1 << bit)) continue;
      const int p2 = p | (1 << bit);
      if (!rv[p2]) continue;
#pragma unroll
      for (int c = 0; c < G; ++c) {
        const double a = x[p][c], b = x[p2][c];
        x[p][c] = a + b;
        x[p2][c] = a - b;
      }
    }
#pragma unroll
    for (int p = 0; p < G; ++p) {  // columns
      if (p & (1 << bit)) continue;
      const int p2 = p | (1 << bit);
      if (!cv[p2] || !two) continue;
#pragma unroll
      for (int r = 0; r < G; ++r) {
        const double a = x[r][p], b = x[r][p2];
        x[r][p] = a + b;
        x[r][p2] = a - b;
      }
    }
#pragma unroll
    for (int r = 0; r < G; ++r)
#pragma unroll
      for (int c = 0; c < G; ++c) x[r][c] *= fr[r] * fc[c];
  }
#pragma unroll
  for (int c = 0; c < G; ++c)
#pragma unroll
    for (int r = 0; r < G; ++r)
      if (rv[r] && cv[c]) {
        if constexpr (STREAM)
          __builtin_nontemporal_store(convert_out<TO>(x[r][c]), &Out[ri[r] + ci[c] * ldo]);
        else
          Out[ri[r] + ci[c] * ldo] = convert_out<TO>(x[r][c]);
      }
}

// One-sided pass on column j of B for the group at rb. op T (U^T b):
// layers hi..lo, mix then scale; op N (V x~): layers lo..hi, scale then mix.
template <int P, int OP, typename PB, typename PC>
__device__ __forceinline__ void transform_vec_block(PB __restrict__ B, int64_t ldb, int64_t j,
                                                    PC __restrict__ C, const Pass &ps,
                                                    int64_t rb) {
  constexpr int G = 1 << P;
  int64_t ri[G];
  bool rv[G];
#pragma unroll
  for (int p = 0; p < G; ++p) {
    ri[p] = rb + p * ps.stride;
    rv[p] = ri[p] < ps.n;
  }
  double x[G];
#pragma unroll
  for (int p = 0; p < G; ++p) x[p] = rv[p] ? B[ri[p] + j * ldb] : 0.0;
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const int bit = (OP == RBT_OP_T) ? s : P - 1 - s;
    const int l = ps.hi - bit;
    const int64_t off = int64_t(l - 1) * ps.n;
    if (ps.rot) {
#pragma unroll
      for (int p = 0; p < G; ++p) {
        if (p & (1 << bit)) continue;
        const int p2 = p | (1 << bit);
        if (!rv[p2]) continue;
        const double c = C[off + ri[p]], sn = C[off + ri[p2]];
        const double a = x[p], b = x[p2];
        x[p] = c * a + sn * b;
        x[p2] = sn * a - c * b;
      }
      continue;
    }
    double f[G];
#pragma unroll
    for (int p = 0; p < G; ++p) {
      const int p2 = p ^ (1 << bit);
      f[p] = rv[p] ? C[off + ri[p]] * ((rv[p2]) ? kInvSqrt2 : 1.0) : 0.0;
    }
    if (OP == RBT_OP_N) {
      // scale by the coefficient of the input index (R_l before O_l); the
      // 1/sqrt(2) of a pair is common to both members, so it can be applied
      // before the mix as well
#pragma unroll
      for (int p = 0; p < G; ++p) x[p] *= f[p];
    }
#pragma unroll
    for (int p = 0; p < G; ++p) {
      if (p & (1 << bit)) continue;
      const int p2 = p | (1 << bit);
      if (!rv[p2]) continue;
      const double a = x[p], b = x[p2];
      x[p] = a + b;
      x[p2] = a - b;
    }
    if (OP == RBT_OP_T) {
#pragma unroll
      for (int p = 0; p < G; ++p) x[p] *= f[p];
    }
  }
#pragma unroll
  for (int p = 0; p < G; ++p)
    if (rv[p]) B[ri[p] + j * ldb] = x[p];
}

}  // namespace dev
}  // namespace rbt

#endif
