// Host-only parts of the ABI: butterfly structure and coefficient draws.
//
// Structure: Sec. 3 (Eq. 2-4) with the loop nest of Algorithm 1 and its
// reference size m = 2^d g ceil(n / (2^d g)) (g = 1: non-tiled; g = n_b:
// tiled, text after Alg. 1; g = lcm(p, q) n_b: Eq. 8). Written here in the closed
// form the kernels use: with q = m / 2^d every index is i = r + t q
// (0 <= r < q, 0 <= t < 2^d); layer l has half-size h_l = 2^(d-l) q, so i is
// in the top half of its layer-l butterfly iff bit (d-l) of t is 0, and its
// partner is i +- h_l when that index is < n.
//
// Coefficients: exp(r/20) with r uniform on [-1, 1) (Sec. 6 setup), from a
// counter-based SplitMix64 (Steele, Lea, Flood, OOPSLA 2014).
#include <cmath>
#include <cstdint>

#include "rbt.h"

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

inline uint64_t splitmix_finalize(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Output number c of SplitMix64 started at state `seed`.
inline uint64_t splitmix_at(uint64_t seed, uint64_t c) {
  return splitmix_finalize(seed + (c + 1) * kGamma);
}

inline double coefficient(uint64_t seed, int side, int layer, int64_t i) {
  const uint64_t c = 128ull * uint64_t(i) + 64ull * uint64_t(side) + uint64_t(layer - 1);
  const double u = double(splitmix_at(seed, c) >> 11) * 0x1.0p-53;
  const double r = 2.0 * u - 1.0;
  return std::exp(r / 20.0);
}

}  // namespace

extern "C" int rbt_version(void) { return 100; }

extern "C" int64_t rbt_reference_size(int64_t n, int depth, int64_t granule) {
  if (n < 0 || depth < 0 || depth > RBT_MAX_DEPTH || granule < 1) return -1;
  const int64_t g = (int64_t(1) << depth) * granule;
  return g * ((n + g - 1) / g);
}

extern "C" int64_t rbt_comm_free_granule(int64_t nb, int64_t p, int64_t q) {
  if (nb < 1 || p < 1 || q < 1) return -1;
  int64_t a = p, b = q;
  while (b != 0) {
    const int64_t t = a % b;
    a = b;
    b = t;
  }
  return (p / a) * q * nb;  // lcm(p, q) nb
}

extern "C" int rbt_structure_ex(int64_t n, int depth, int64_t granule, int64_t *partner) {
  if (n < 0) return -1;
  if (depth < 0 || depth > RBT_MAX_DEPTH) return -2;
  if (granule < 1) return -3;
  if (partner == nullptr && n > 0 && depth > 0) return -4;
  const int64_t m = rbt_reference_size(n, depth, granule);
  const int64_t q = (n == 0) ? 1 : (m >> depth);
  for (int layer = 1; layer <= depth; ++layer) {
    const int64_t bit = int64_t(1) << (depth - layer);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t r = i % q, t = i / q;
      const int64_t j = r + (t ^ bit) * q;
      partner[int64_t(layer - 1) * n + i] = (j < n) ? j : -1;
    }
  }
  return 0;
}

extern "C" int rbt_structure(int64_t n, int depth, int64_t *partner) {
  const int rc = rbt_structure_ex(n, depth, 1, partner);
  return rc == -4 ? -3 : rc;
}

// Rotation butterflies: cos(theta) at the top index of a pair, sin(theta) at
// the bottom one, 1 where unpaired; theta = 2 pi u from the counter of the
// pair's top index.
extern "C" int rbt_generate_rotations(int64_t n, int depth, uint64_t seed, int64_t granule,
                                      double *U, double *V) {
  if (n < 0) return -1;
  if (depth < 0 || depth > RBT_MAX_DEPTH) return -2;
  if (granule < 1) return -4;
  if (U == nullptr && n > 0 && depth > 0) return -5;
  if (V == nullptr && n > 0 && depth > 0) return -6;
  const int64_t m = rbt_reference_size(n, depth, granule);
  const int64_t q = (n == 0) ? 1 : (m >> depth);
  for (int side = 0; side < 2; ++side) {
    double *C = side ? V : U;
    for (int layer = 1; layer <= depth; ++layer) {
      const int64_t bit = int64_t(1) << (depth - layer);
      for (int64_t i = 0; i < n; ++i) {
        const int64_t r = i % q, t = i / q;
        const int64_t j = r + (t ^ bit) * q;
        double v = 1.0;
        if (j < n) {
          const bool top = (t & bit) == 0;
          const int64_t a = top ? i : j;
          const uint64_t c = 128ull * uint64_t(a) + 64ull * uint64_t(side) + uint64_t(layer - 1);
          const double u = double(splitmix_at(seed, c) >> 11) * 0x1.0p-53;
          const double th = 2.0 * 3.14159265358979323846 * u;
          v = top ? std::cos(th) : std::sin(th);
        }
        C[int64_t(layer - 1) * n + i] = v;
      }
    }
  }
  return 0;
}

extern "C" int rbt_generate(int64_t n, int depth, uint64_t seed, double *U, double *V) {
  if (n < 0) return -1;
  if (depth < 0 || depth > RBT_MAX_DEPTH) return -2;
  if (U == nullptr && n > 0 && depth > 0) return -4;
  if (V == nullptr && n > 0 && depth > 0) return -5;
  for (int layer = 1; layer <= depth; ++layer) {
    for (int64_t i = 0; i < n; ++i) {
      U[int64_t(layer - 1) * n + i] = coefficient(seed, 0, layer, i);
      V[int64_t(layer - 1) * n + i] = coefficient(seed, 1, layer, i);
    }
  }
  return 0;
}
