// Batched solves of many independent systems of different sizes in ONE
// persistent launch: each workgroup takes systems from a queue (largest
// first, as ordered by the host plan) and runs the whole method on each:
// coefficients (Sec. 6 law), the two-sided transform A~ = U^T A V stored in
// FP32 (Eq. 1), elimination without pivoting in FP32 (or with BF16 trailing
// update operands), the solve of Eq. 1 with the low-precision factors, and
// FP64 refinement with the original A until the Eq. 7 backward error is
// <= tol (Sec. 5).
//
// Per system, in the workspace: F (n x n FP32, ld n) holds A~ and then its
// L\U factors; the FP64 area holds U, V (n x d each), the inverses of the
// 64 x 64 diagonal blocks (strictly lower part: L^-1, upper part with the
// diagonal: U^-1, one 64 x 64 array per block, in the factors' type) and
// the residual (n x nrhs); the fallback area holds FP64 factors.
//
// Elimination, per 64-column step k (right-looking), in the factors'
// arithmetic type (FP32 for the low-precision pass, FP64 for the fallback):
//   diagonal block in LDS: 16-column panels factored by wavefront 0 with
//   readlane broadcasts, U rows by substitution, rank-16 updates; its
//   inverses L^-1 and U^-1 by substitution (one column per lane: wavefront
//   0 the columns of L^-1, wavefront 1 those of U^-1);
//   L21 = A21 U11^-1 and U12 = L11^-1 A12 as matrix-core products with the
//   inverses (FP32: plus one refinement step, X += (A - X D) D^-1), and
//   A22 -= L21 U12 (FP32: v_mfma_f32_16x16x4f32, or BF16 operands on
//   v_mfma_f32_16x16x32_bf16), all in 64 x 64 tiles.
// Solves: block sweeps over the factors with the inverses of the diagonal
// blocks (FP32: plus one refinement step per block).
//
// The host plan (rbt_batched_plan) writes the header and the descriptor
// table; the kernel checks the header against its arguments and does
// nothing for a plan that does not match.
#include "butterfly_dev.h"
#include "mma16.h"

namespace rbt {

namespace {

constexpr int BT = 256;      // threads per workgroup
constexpr int BB = 64;       // block size of the per-system elimination
constexpr int LDS_ = BB + 1; // LDS leading dimension of FP64 64 x 64 blocks
constexpr int LDF = BB + 1;  // FP32 tiles
constexpr int LDH = BB + 8;  // BF16 tiles (rows of 144 bytes)
constexpr int NR = kSkinnyMax;  // right-hand sides per system, at most

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// Global-memory pointers: the phase functions below are not inlined and
// reach the factor storage through Sys, so the compiler cannot tell that it
// is global memory and would use FLAT instructions, which also count against
// the LDS counter (every wait for LDS data in the MFMA loop would then wait
// for the prefetched global loads). The pipelined trailing update therefore
// casts its pointers to the global address space explicitly.
#define RBT_AS_GLOBAL __attribute__((address_space(1)))
typedef float RBT_AS_GLOBAL gfloat;
// The same for LDS pointers that reach a non-inlined function as
// arguments: with the address space explicit, LDS accesses are plain ds
// instructions on 32-bit addresses (no generic-to-LDS conversion per
// access) and loads from valid LDS addresses can be issued unconditionally.
#define RBT_AS_LDS __attribute__((address_space(3)))
typedef double RBT_AS_LDS ldouble;
// LDS pointer of element type C
template <typename C>
struct Lds {
  typedef C RBT_AS_LDS T;
};
__device__ __forceinline__ f4u ld4(const float *p) { return *reinterpret_cast<const f4u *>(p); }
__device__ __forceinline__ f4u ld4(const gfloat *p) {
  return *reinterpret_cast<const f4u RBT_AS_GLOBAL *>(p);
}
__device__ __forceinline__ void st4(float *p, f4u v) { *reinterpret_cast<f4u *>(p) = v; }
__device__ __forceinline__ void st4(gfloat *p, f4u v) {
  *reinterpret_cast<f4u RBT_AS_GLOBAL *>(p) = v;
}


// LDS: region 0 (the diagonal block S, or the GEMM tiles, or the residual
// buffers) and region 1 (the inverses T, kept through the panel products of
// a step); the sweeps use both regions.
constexpr int kR0Doubles = BB * LDS_;       // 4160 doubles
constexpr int kR1Doubles = BB * LDS_;
static_assert(7 * BB * NR <= kR0Doubles + kR1Doubles, "sweep buffers exceed LDS");  // part, xs, ys, x0s
static_assert(256 * NR + BT / 64 <= kR0Doubles, "residual buffers exceed region 0");

struct Args {
  int64_t batch;
  char *work;
  size_t work_bytes;
  const double *const *A;
  const int64_t *lda;
  const double *const *B;
  const int64_t *ldb;
  double *const *X;
  const int64_t *ldx;
  int32_t *iters;
  double *berr;
  int32_t *info;
  int32_t *path;
  uint64_t seed;
  double tol;
  int depth, prec, max_iter;
  int64_t granule;  // reference-size granule of the butterfly structure
  int kind, sides;  // butterfly kind (1: rotations) and sides (1: one-sided)
  int64_t ct2_min_n;  // systems with n >= this: two 64-column tiles per round
};

// A value that is the same in every lane, moved to scalar registers: the
// phase functions below are not inlined and read sizes, strides and base
// pointers through Sys, so the compiler cannot tell they are uniform and
// would keep them (and every address formed from them) in vector registers.
__device__ __forceinline__ int64_t wave_uniform(int64_t v) {
  const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v))));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(uint64_t(v) >> 32))));
  return int64_t((uint64_t(hi) << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T *wave_uniform(T *p) {
  return reinterpret_cast<T *>(wave_uniform(int64_t(reinterpret_cast<uintptr_t>(p))));
}

__device__ __forceinline__ double nanmax(double a, double b) {
  return (b > a || b != b) ? b : a;
}

// NaN-propagating maximum over the workgroup (red: BT/64 doubles of LDS).
__device__ double wg_nanmax(double v, double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = nanmax(v, __shfl_xor(v, o));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int w = 1; w < BT / 64; ++w) r = nanmax(r, red[w]);
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------- tiles

// acc (per wavefront 32 x 32 of a 64 x 64 tile) = A (64 x K) B (K x 64),
// K = 64, operands staged in LDS: FP32 As[m][k], Bs[n][k] (ld LDF) or BF16
// Ah[m][k], Bh[n][k] (ld LDH).
template <bool BF16>
__device__ __forceinline__ void tile_mma(const void *sa, const void *sb, f4 (&acc)[2][2]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int l16 = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  if constexpr (!BF16) {
    const float(*As)[LDF] = reinterpret_cast<const float(*)[LDF]>(sa);
    const float(*Bs)[LDF] = reinterpret_cast<const float(*)[LDF]>(sb);
#pragma unroll
    for (int kk = 0; kk < BB / 4; ++kk) {
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[wm * 32 + 16 * i + l16][4 * kk + lk];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[wn * 32 + 16 * j + l16][4 * kk + lk];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  } else {
    const __bf16(*Ah)[LDH] = reinterpret_cast<const __bf16(*)[LDH]>(sa);
    const __bf16(*Bh)[LDH] = reinterpret_cast<const __bf16(*)[LDH]>(sb);
#pragma unroll
    for (int kk = 0; kk < BB / 32; ++kk) {
      bf8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        a[i] = *reinterpret_cast<const bf8 *>(&Ah[wm * 32 + 16 * i + l16][32 * kk + 8 * lk]);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        b[j] = *reinterpret_cast<const bf8 *>(&Bh[wn * 32 + 16 * j + l16][32 * kk + 8 * lk]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
}

// Stage a 64 x 64 operand in LDS as dst[r][k] from a column-major FP32
// source whose element (r, k) is src[r + k * ld] (rmode: r runs down a
// column) or src[k + r * ld] (kmode: k runs down a column). Entries with
// r >= rv or k >= kv are zero.
template <bool BF16, bool KMODE, typename PF>
__device__ __forceinline__ void stage(void *dst, PF src, int64_t ld, int rv, int kv) {
  const int tid = threadIdx.x;
  // thread: column c = tid / 4 of the source, 16 consecutive entries
  const int col = tid >> 2, seg = (tid & 3) * 16;
  float v[16];
  if (KMODE) {
    // source column = operand row r = col; entries k = seg..seg+15
    const bool full = col < rv && seg + 16 <= kv;
    const PF p = src + seg + int64_t(col) * ld;
    if (full) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f4u t = ld4(p + 4 * q);
        v[4 * q] = t[0]; v[4 * q + 1] = t[1]; v[4 * q + 2] = t[2]; v[4 * q + 3] = t[3];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) v[e] = (col < rv && seg + e < kv) ? p[e] : 0.0f;
    }
    if constexpr (BF16) {
      __bf16(*D)[LDH] = reinterpret_cast<__bf16(*)[LDH]>(dst);
#pragma unroll
      for (int e = 0; e < 16; ++e) D[col][seg + e] = (__bf16)v[e];
    } else {
      float(*D)[LDF] = reinterpret_cast<float(*)[LDF]>(dst);
#pragma unroll
      for (int e = 0; e < 16; ++e) D[col][seg + e] = v[e];
    }
  } else {
    // source column = operand k = col; entries r = seg..seg+15
    const bool full = col < kv && seg + 16 <= rv;
    const PF p = src + seg + int64_t(col) * ld;
    if (full) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f4u t = ld4(p + 4 * q);
        v[4 * q] = t[0]; v[4 * q + 1] = t[1]; v[4 * q + 2] = t[2]; v[4 * q + 3] = t[3];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) v[e] = (col < kv && seg + e < rv) ? p[e] : 0.0f;
    }
    if constexpr (BF16) {
      __bf16(*D)[LDH] = reinterpret_cast<__bf16(*)[LDH]>(dst);
#pragma unroll
      for (int e = 0; e < 16; ++e) D[seg + e][col] = (__bf16)v[e];
    } else {
      float(*D)[LDF] = reinterpret_cast<float(*)[LDF]>(dst);
#pragma unroll
      for (int e = 0; e < 16; ++e) D[seg + e][col] = v[e];
    }
  }
}

// Apply a tile result to C (column-major FP32, ld): rows r0.., cols c0..,
// valid rv x cv; SUB: C -= acc, else C = acc.
template <bool SUB>
__device__ __forceinline__ void tile_store(const f4 (&acc)[2][2], float *C, int64_t ld, int rv,
                                           int cv) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int l16 = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = wn * 32 + 16 * j + l16;
      if (col >= cv) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wm * 32 + 16 * i + 4 * lk + v;
        if (row < rv) {
          float *p = C + row + int64_t(col) * ld;
          if (SUB)
            *p -= acc[i][j][v];
          else
            *p = acc[i][j][v];
        }
      }
    }
}

// Register stages of the pipelined trailing update (A22 -= L21 U12): the
// next U12 tile and the next C tile are loaded into registers while the
// matrix cores work on the current tile.
// U12 tile (kv x cv, element (kx, nx) at src[kx + nx * ld]): thread holds
// operand row nx = tid / 4, entries kx = 16 (tid % 4) + 0..15 (zero outside).
template <typename PF>
__device__ __forceinline__ void load_bt(float (&v)[16], PF src, int64_t ld, int cv, int kv) {
  const int tid = threadIdx.x;
  const int col = tid >> 2, seg = (tid & 3) * 16;
  const PF p = src + seg + int64_t(col) * ld;
  if (col < cv && seg + 16 <= kv) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const f4u t = ld4(p + 4 * q);
      v[4 * q] = t[0]; v[4 * q + 1] = t[1]; v[4 * q + 2] = t[2]; v[4 * q + 3] = t[3];
    }
  } else {
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = (col < cv && seg + e < kv) ? p[e] : 0.0f;
  }
}
template <bool BF16>
__device__ __forceinline__ void store_bt(void *dst, const float (&v)[16]) {
  const int tid = threadIdx.x;
  const int col = tid >> 2, seg = (tid & 3) * 16;
  if constexpr (BF16) {
    __bf16(*D)[LDH] = reinterpret_cast<__bf16(*)[LDH]>(dst);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      bf8 w;
#pragma unroll
      for (int e = 0; e < 8; ++e) w[e] = (__bf16)v[8 * h + e];
      *reinterpret_cast<bf8 *>(&D[col][seg + 8 * h]) = w;
    }
  } else {
    float(*D)[LDF] = reinterpret_cast<float(*)[LDF]>(dst);
#pragma unroll
    for (int e = 0; e < 16; ++e) D[col][seg + e] = v[e];
  }
}
// C tile (rv x cv at C, column-major ld) in the accumulator layout of
// tile_mma: (i, j, v) is row wm*32 + 16 i + 4 (lane/16) + v, column
// wn*32 + 16 j + lane%16. Entries outside the tile read as zero and are not
// written.
template <typename PF>
__device__ __forceinline__ void load_ct(f4 (&c)[2][2], PF C, int64_t ld, int rv, int cv) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int l16 = lane & 15, lk = lane >> 4;
  const bool full = rv == BB && cv == BB;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int row = wm * 32 + 16 * i + 4 * lk, col = wn * 32 + 16 * j + l16;
      const PF p = C + row + int64_t(col) * ld;
      if (full) {
        const f4u t = ld4(p);
        c[i][j] = f4{t[0], t[1], t[2], t[3]};
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) c[i][j][v] = (col < cv && row + v < rv) ? p[v] : 0.0f;
      }
    }
}
template <typename PF>
__device__ __forceinline__ void store_ct(const f4 (&c)[2][2], PF C, int64_t ld, int rv, int cv) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int l16 = lane & 15, lk = lane >> 4;
  const bool full = rv == BB && cv == BB;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int row = wm * 32 + 16 * i + 4 * lk, col = wn * 32 + 16 * j + l16;
      const PF p = C + row + int64_t(col) * ld;
      if (full) {
        st4(p, f4u{c[i][j][0], c[i][j][1], c[i][j][2], c[i][j][3]});
      } else if (col < cv) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (row + v < rv) p[v] = c[i][j][v];
      }
    }
}

// Panel products (the solves with the diagonal block's inverses) on the
// 16 x 16 x 4 matrix cores of the factors' arithmetic type C (FP32 for the
// low-precision pass, FP64 for the fallback; mma16.h gives the output
// layout). Operands come from accessors a(m, k), b(k, n); acc is one
// wavefront's 32 x 32 part of a 64 x 64 tile, K = 64.
template <typename C, typename FA, typename FB>
__device__ __forceinline__ void tile_mma_c(FA a_at, FB b_at, typename Mma16<C>::v4 (&acc)[2][2]) {
  typedef typename Mma16<C>::v4 c4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int l16 = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = c4{C(0), C(0), C(0), C(0)};
#pragma unroll 4
  for (int kk = 0; kk < BB / 4; ++kk) {
    C a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = a_at(wm * 32 + 16 * i + l16, 4 * kk + lk);
#pragma unroll
    for (int j = 0; j < 2; ++j) b[j] = b_at(4 * kk + lk, wn * 32 + 16 * j + l16);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = Mma16<C>::mma(a[i], b[j], acc[i][j]);
  }
}

// Cm (FP32 or FP64, ld) = acc, or Cm -= acc (SUB), in type C; rows < rv,
// cols < cv.
template <typename C, bool SUB = false, typename T>
__device__ __forceinline__ void tile_store_c(const typename Mma16<C>::v4 (&acc)[2][2], T *Cm,
                                             int64_t ld, int rv, int cv) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int l16 = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = wn * 32 + 16 * j + l16;
      if (col >= cv) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wm * 32 + 16 * i + Mma16<C>::row(lk, v);
        if (row < rv) {
          T RBT_AS_GLOBAL *p = (T RBT_AS_GLOBAL *)Cm + row + int64_t(col) * ld;
          if (SUB)
            *p = T(C(*p) - acc[i][j][v]);
          else
            *p = T(acc[i][j][v]);
        }
      }
    }
}

template <typename C>
__device__ __forceinline__ void add_acc(typename Mma16<C>::v4 (&a)[2][2],
                                        const typename Mma16<C>::v4 (&b)[2][2]) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) a[i][j] += b[i][j];
}

// D[col * LDS_ + row] = acc (SUB: D -= acc) for the tile elements of this
// lane (LDS, type C, all 64 x 64 entries).
template <typename C, bool SUB = false>
__device__ __forceinline__ void tile_to_lds(const typename Mma16<C>::v4 (&acc)[2][2],
                                            typename Lds<C>::T *D) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int l16 = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = wn * 32 + 16 * j + l16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wm * 32 + 16 * i + Mma16<C>::row(lk, v);
        if (SUB)
          D[col * LDS_ + row] -= acc[i][j][v];
        else
          D[col * LDS_ + row] = acc[i][j][v];
      }
    }
}

// Stage a 64 x 64 block of F (FP32 or FP64, column-major, rows r0..,
// cols c0..; rv x cv valid) in LDS as D[c * LDS_ + r] of type C (zero
// outside). (src is factor storage, D is LDS: both address spaces made
// explicit.)
template <typename C, typename T>
__device__ __forceinline__ void stage_c(C *D_in, const T *src_in, int64_t ld, int rv, int cv) {
  typename Lds<C>::T *D = (typename Lds<C>::T *)D_in;
  const T RBT_AS_GLOBAL *src = (const T RBT_AS_GLOBAL *)src_in;
  const int tid = threadIdx.x;
  const int col = tid >> 2, seg = (tid & 3) * 16;
  T v[16];
  if constexpr (sizeof(T) == 4) {
    if (col < cv && seg + 16 <= rv) {
      const gfloat *p = src + seg + int64_t(col) * ld;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f4u t = ld4(p + 4 * q);
        v[4 * q] = t[0]; v[4 * q + 1] = t[1]; v[4 * q + 2] = t[2]; v[4 * q + 3] = t[3];
      }
    } else {
      const T RBT_AS_GLOBAL *p = src + int64_t(col < cv ? col : 0) * ld;
#pragma unroll
      for (int e = 0; e < 16; ++e) v[e] = (col < cv && seg + e < rv) ? p[seg + e] : T(0);
    }
  } else {
    const T RBT_AS_GLOBAL *p = src + int64_t(col < cv ? col : 0) * ld;
    const int rl = rv - 1;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const T x = p[seg + e < rv ? seg + e : (rl > 0 ? rl : 0)];
      v[e] = (col < cv && seg + e < rv) ? x : T(0);
    }
  }
#pragma unroll
  for (int e = 0; e < 16; ++e) D[col * LDS_ + seg + e] = C(v[e]);
}

// ------------------------------------------------------- one system

struct Sys {
  int64_t n, nrhs;
  int64_t q;         // m / 2^d of the butterfly structure
  int rot, sides;    // butterfly kind (rotations) and sides
  float *F;          // n x n, ld n
  double *F64;       // n x n, ld n: FP64 factors of the fallback (nullable)
  double *U, *V;     // n x d each
  double *Inv;       // nblk x 64 x 64
  double *R;         // n x nrhs
  const double *A;
  int64_t lda;
  const double *Bm;
  int64_t ldb;
  double *Xm;
  int64_t ldx;
};

template <typename T>
__device__ __forceinline__ T *fmat(const Sys &s) {
  if constexpr (sizeof(T) == 4)
    return wave_uniform(s.F);
  else
    return wave_uniform(s.F64);
}

// Factor the kb x kb diagonal block at (k, k) of F in the factors'
// arithmetic type TF (FP32 for the low-precision pass, FP64 for the
// fallback): S (LDS) <- L\U, T (LDS) <- L^-1 below the diagonal, U^-1 on
// and above; inverses also to Inv (64 x 64 of type TF, full, identity beyond
// kb); factors back to F.
template <typename TF>
__device__ __noinline__ void diag_block(const Sys &s, int64_t k, int kb, double *S_in, double *T_in,
                                        TF *Invb, int *info_sh) {
  typedef typename Lds<TF>::T lds_t;
  lds_t *S = (lds_t *)S_in;
  lds_t *T = (lds_t *)T_in;
  TF RBT_AS_GLOBAL *F = (TF RBT_AS_GLOBAL *)fmat<TF>(s);
  TF RBT_AS_GLOBAL *Invg = (TF RBT_AS_GLOBAL *)wave_uniform(Invb);
  const int64_t n = wave_uniform(s.n);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  {
    const int r = tid & 63, cg = tid >> 6;
    const int rr = r < kb ? r : kb - 1;
    TF v[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int c = cg + 4 * t;
      v[t] = F[(k + rr) + (k + (c < kb ? c : kb - 1)) * n];
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int c = cg + 4 * t;
      S[c * LDS_ + r] = (r < kb && c < kb) ? v[t] : (r == c ? TF(1) : TF(0));
    }
  }
  __syncthreads();
  for (int c0 = 0; c0 < BB; c0 += 16) {
    if (wave == 0) {
      TF xa[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) xa[j] = S[(c0 + j) * LDS_ + lane];
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) {
        const int c = c0 + cc;
        TF prow[16];
#pragma unroll
        for (int j = cc; j < 16; ++j) prow[j] = wave_bcast(xa[j], c);
        const TF p = prow[cc];
        if (lane == 0 && c < kb && p == TF(0) && *info_sh == 0) *info_sh = int(k + c + 1);
        const bool act = lane > c;
        // one division per pivot; rows above it take a zero multiplier
        const TF la = act ? xa[cc] * (TF(1) / p) : TF(0);
        xa[cc] = act ? la : xa[cc];
#pragma unroll
        for (int j = cc + 1; j < 16; ++j) xa[j] -= la * prow[j];
      }
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (lane >= c0) S[(c0 + j) * LDS_ + lane] = xa[j];
    }
    __syncthreads();
    const int c1 = c0 + 16;
    if (c1 >= BB) break;
    if (tid < BB - c1) {  // U rows c0..c0+15, columns c1..63
      const int col = c1 + tid;
      TF y[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) y[i] = S[col * LDS_ + c0 + i];
#pragma unroll
      for (int i = 0; i < 16; ++i)
#pragma unroll
        for (int i2 = i + 1; i2 < 16; ++i2) y[i2] -= S[(c0 + i) * LDS_ + c0 + i2] * y[i];
#pragma unroll
      for (int i = 0; i < 16; ++i) S[col * LDS_ + c0 + i] = y[i];
    }
    __syncthreads();
    const int w = BB - c1;
    for (int e = tid; e < w * w; e += BT) {
      const int i = c1 + e % w, j = c1 + e / w;
      TF a = S[j * LDS_ + i];
#pragma unroll
      for (int t = 0; t < 16; ++t) a -= S[(c0 + t) * LDS_ + i] * S[j * LDS_ + c0 + t];
      S[j * LDS_ + i] = a;
    }
    __syncthreads();
  }
  // inverses, lane c of a wavefront owning column c (its own column of T,
  // so no barriers): wave 0 L^-1 (strictly lower part of T), wave 1 U^-1
  // (upper part with the diagonal). Rows are taken in a uniform order (L:
  // top-down, U: bottom-up), so the factor entry of a step is one broadcast
  // LDS read and the sum over the solved rows has a uniform range (masked
  // per lane), unrolled into independent partial sums.
  if (wave == 0) {
    const int c = lane;
    for (int i = 1; i < BB; ++i) {  // X[i][c] = -(L[i][c] + sum_{c<t<i} L[i][t] X[t][c]), i > c
      TF p0 = TF(0), p1 = TF(0), p2 = TF(0), p3 = TF(0);
      int t = 0;
      for (; t + 4 <= i; t += 4) {
        const TF t0 = T[c * LDS_ + t + 0], t1 = T[c * LDS_ + t + 1];
        const TF t2 = T[c * LDS_ + t + 2], t3 = T[c * LDS_ + t + 3];
        const TF x0 = t + 0 > c ? t0 : (t + 0 == c ? TF(1) : TF(0));
        const TF x1 = t + 1 > c ? t1 : (t + 1 == c ? TF(1) : TF(0));
        const TF x2 = t + 2 > c ? t2 : (t + 2 == c ? TF(1) : TF(0));
        const TF x3 = t + 3 > c ? t3 : (t + 3 == c ? TF(1) : TF(0));
        p0 += S[(t + 0) * LDS_ + i] * x0;
        p1 += S[(t + 1) * LDS_ + i] * x1;
        p2 += S[(t + 2) * LDS_ + i] * x2;
        p3 += S[(t + 3) * LDS_ + i] * x3;
      }
      for (; t < i; ++t) {
        const TF tv = T[c * LDS_ + t];
        const TF x = t > c ? tv : (t == c ? TF(1) : TF(0));
        p0 += S[t * LDS_ + i] * x;
      }
      if (i > c) T[c * LDS_ + i] = -((p0 + p1) + (p2 + p3));
    }
  } else if (wave == 1) {
    const int c = lane;
    T[c * LDS_ + c] = TF(1) / S[c * LDS_ + c];
    for (int i = BB - 2; i >= 0; --i) {  // X[i][c] = -(sum_{i<t<=c} U[i][t] X[t][c]) / U[i][i], i < c
      const TF rd = TF(1) / S[i * LDS_ + i];
      TF p0 = TF(0), p1 = TF(0), p2 = TF(0), p3 = TF(0);
      int t = i + 1;
      for (; t + 4 <= BB; t += 4) {
        const TF t0 = T[c * LDS_ + t + 0], t1 = T[c * LDS_ + t + 1];
        const TF t2 = T[c * LDS_ + t + 2], t3 = T[c * LDS_ + t + 3];
        const TF x0 = t + 0 <= c ? t0 : TF(0);
        const TF x1 = t + 1 <= c ? t1 : TF(0);
        const TF x2 = t + 2 <= c ? t2 : TF(0);
        const TF x3 = t + 3 <= c ? t3 : TF(0);
        p0 += S[(t + 0) * LDS_ + i] * x0;
        p1 += S[(t + 1) * LDS_ + i] * x1;
        p2 += S[(t + 2) * LDS_ + i] * x2;
        p3 += S[(t + 3) * LDS_ + i] * x3;
      }
      for (; t < BB; ++t) {
        const TF tv = T[c * LDS_ + t];
        const TF x = t <= c ? tv : TF(0);
        p0 += S[t * LDS_ + i] * x;
      }
      if (i < c) T[c * LDS_ + i] = -((p0 + p1) + (p2 + p3)) * rd;
    }
  }
  __syncthreads();
  // FP32: a copy of L\U (identity beyond kb) in the second half of region 1
  // for the refinement step of the panel products
  lds_t *Sc = T + BB * LDS_;
  for (int e = tid; e < BB * BB; e += BT) {
    const int r = e & 63, c = e >> 6;
    Invg[r + c * BB] = T[c * LDS_ + r];
    if (r < kb && c < kb) F[(k + r) + (k + c) * n] = S[c * LDS_ + r];
    if constexpr (sizeof(TF) == 4) Sc[c * LDS_ + r] = S[c * LDS_ + r];
  }
  __syncthreads();
}

// TF = float: FP32 factors (trailing update in FP32 or, BF16U, with BF16
// operands; CT column tiles of 64 per round of the trailing update);
// TF = double: FP64 factors (the fallback; FP64 trailing update).
template <typename TF, bool BF16U, int CT = 1>
__device__ __noinline__ void eliminate(const Sys &s, double *L0, double *L1, int *info_sh) {
  const int64_t n = wave_uniform(s.n);
  TF *F = fmat<TF>(s);
  TF *Inv = reinterpret_cast<TF *>(wave_uniform(s.Inv));
  float(*As)[LDF] = reinterpret_cast<float(*)[LDF]>(L0);
  float(*Bs)[LDF] = reinterpret_cast<float(*)[LDF]>(L0 + (BB * LDF + 1) / 2);
  __bf16(*Ah)[LDH] = reinterpret_cast<__bf16(*)[LDH]>(L0);
  __bf16(*Bh)[LDH] = reinterpret_cast<__bf16(*)[LDH]>(L0 + (BB * LDH) / 4);
  for (int64_t k = 0; k < n; k += BB) {
    const int kb = int(n - k < BB ? n - k : BB);
    // inverse block k / BB, counted in elements of the factors' type (the
    // sweeps index the area the same way)
    TF *Invb = Inv + (k / BB) * BB * BB;
    diag_block<TF>(s, k, kb, L0, L1, Invb, info_sh);
    const int64_t rest = n - k - kb;
    if (rest <= 0) break;
    f4 acc[2][2];
    typename Mma16<double>::v4 acc64[2][2];
    // panel products in the factors' arithmetic type. A product with an
    // explicit inverse of the diagonal block is accurate to kappa(block) u
    // only; in FP32 that is too coarse for refinement to converge on
    // high-growth N(0,1) systems, so the FP32 products take one
    // refinement step (region 0 holds the staged panel tile and the first
    // product, region 1 the inverses and a copy of L\U). The FP64 factors
    // of the fallback use the inverses alone (kappa u64 is small).
    constexpr bool kRefinePanel = sizeof(TF) == 4;
    typename Mma16<TF>::v4 accp[2][2], accq[2][2];
    typedef typename Lds<TF>::T lds_t;
    const lds_t *T = (const lds_t *)L1;  // L^-1 below the diagonal, U^-1 on and above (ld LDS_)
    const lds_t *Sc = T + BB * LDS_;     // FP32: L\U of the diagonal block
    const lds_t *L0l = (const lds_t *)L0;
    lds_t *L0w = (lds_t *)L0;
    lds_t *X0s = L0w + BB * LDS_;        // FP32: the first product
    TF *L0t = reinterpret_cast<TF *>(L0);
    // L21 = A21 U11^-1 (rows k+kb.., 64-row tiles)
    for (int64_t r0 = k + kb; r0 < n; r0 += BB) {
      const int rv = int(n - r0 < BB ? n - r0 : BB);
      // stage A21 tile as [k][r]: element (r, kx) at L0[kx * LDS_ + r]
      stage_c<TF>(L0t, F + r0 + k * n, n, rv, kb);
      __syncthreads();
      auto uinv = [&](int kx, int nx) { return kx <= nx ? T[nx * LDS_ + kx] : TF(0); };
      tile_mma_c<TF>([&](int m, int kx) { return L0l[kx * LDS_ + m]; }, uinv, accp);
      if constexpr (kRefinePanel) {
        // one refinement step: R = A21 - X U11 (over the staged A21), then
        // X += R U11^-1
        tile_to_lds<TF>(accp, X0s);
        __syncthreads();
        tile_mma_c<TF>([&](int m, int kx) { return X0s[kx * LDS_ + m]; },
                       [&](int kx, int nx) { return kx <= nx ? Sc[nx * LDS_ + kx] : TF(0); }, accq);
        tile_to_lds<TF, true>(accq, L0w);
        __syncthreads();
        tile_mma_c<TF>([&](int m, int kx) { return L0l[kx * LDS_ + m]; }, uinv, accq);
        add_acc<TF>(accp, accq);
      }
      __syncthreads();
      tile_store_c<TF>(accp, F + r0 + k * n, n, rv, kb);
    }
    __syncthreads();
    // U12 = L11^-1 A12 (64-column tiles)
    for (int64_t c0 = k + kb; c0 < n; c0 += BB) {
      const int cv = int(n - c0 < BB ? n - c0 : BB);
      // stage A12 tile: element (kx, nx) at L0[nx * LDS_ + kx]
      stage_c<TF>(L0t, F + k + c0 * n, n, kb, cv);
      __syncthreads();
      auto linv = [&](int m, int kx) {
        return m > kx ? T[kx * LDS_ + m] : (m == kx ? TF(1) : TF(0));
      };
      tile_mma_c<TF>(linv, [&](int kx, int nx) { return L0l[nx * LDS_ + kx]; }, accp);
      if constexpr (kRefinePanel) {
        // R = A12 - L11 X (over the staged A12), then X += L11^-1 R
        tile_to_lds<TF>(accp, X0s);
        __syncthreads();
        tile_mma_c<TF>(
            [&](int m, int kx) { return m > kx ? Sc[kx * LDS_ + m] : (m == kx ? TF(1) : TF(0)); },
            [&](int kx, int nx) { return X0s[nx * LDS_ + kx]; }, accq);
        tile_to_lds<TF, true>(accq, L0w);
        __syncthreads();
        tile_mma_c<TF>(linv, [&](int kx, int nx) { return L0l[nx * LDS_ + kx]; }, accq);
        add_acc<TF>(accp, accq);
      }
      __syncthreads();
      tile_store_c<TF>(accp, F + k + c0 * n, n, kb, cv);
    }
    __syncthreads();
    // A22 -= L21 U12 (64 x 64 tiles; the L21 row tile stays in LDS)
    if constexpr (sizeof(TF) == 4) {
      // low precision: CT column tiles per round (the second U12 tile in
      // region 1, free after the panel products); the next round's U12 and
      // C tiles are loaded into registers while the matrix cores work
      gfloat *Fg = (gfloat *)F;
      void *bdst[CT];
      bdst[0] = BF16U ? static_cast<void *>(Bh) : static_cast<void *>(Bs);
      if constexpr (CT > 1) bdst[1] = static_cast<void *>(L1);
      for (int64_t r0 = k + kb; r0 < n; r0 += BB) {
        const int rv = int(n - r0 < BB ? n - r0 : BB);
        if constexpr (BF16U)
          stage<true, false>(Ah, Fg + r0 + k * n, n, rv, kb);
        else
          stage<false, false>(As, Fg + r0 + k * n, n, rv, kb);
        float bv[CT][16];
        f4 cn[CT][2][2];
        auto prefetch = [&](int64_t cbase) {
#pragma unroll
          for (int t = 0; t < CT; ++t) {
            const int64_t c = cbase + int64_t(t) * BB;
            if (c < n) {
              const int cv = int(n - c < BB ? n - c : BB);
              load_bt(bv[t], Fg + k + c * n, n, cv, kb);
              load_ct(cn[t], Fg + r0 + c * n, n, rv, cv);
            }
          }
        };
        prefetch(k + kb);
        for (int64_t c0 = k + kb; c0 < n; c0 += CT * BB) {
          f4 cc[CT][2][2];
#pragma unroll
          for (int t = 0; t < CT; ++t) {
            if (c0 + int64_t(t) * BB < n) store_bt<BF16U>(bdst[t], bv[t]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int j = 0; j < 2; ++j) cc[t][i][j] = cn[t][i][j];
          }
          __syncthreads();
          prefetch(c0 + CT * BB);
#pragma unroll
          for (int t = 0; t < CT; ++t) {
            const int64_t c = c0 + int64_t(t) * BB;
            if (c >= n) break;
            const int cv = int(n - c < BB ? n - c : BB);
            if constexpr (BF16U)
              tile_mma<true>(Ah, bdst[t], acc);
            else
              tile_mma<false>(As, bdst[t], acc);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int j = 0; j < 2; ++j) cc[t][i][j] -= acc[i][j];
            store_ct(cc[t], Fg + r0 + c * n, n, rv, cv);
          }
          __syncthreads();
        }
      }
      __syncthreads();
      continue;
    }
    // FP64 factors (the fallback): the same pipeline with FP64 tiles; the
    // L21 row tile stays in L0, the U12 tile goes through L1
    double RBT_AS_GLOBAL *Fd = (double RBT_AS_GLOBAL *)F;
    ldouble *L0d = (ldouble *)L0, *L1d = (ldouble *)L1;
    const int tid = threadIdx.x;
    const int bcol = tid >> 2, bseg = (tid & 3) * 16;  // U12 tile: column nx, rows kx
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1, l16 = lane & 15, lk = lane >> 4;
    for (int64_t r0 = k + kb; r0 < n; r0 += BB) {
      const int rv = int(n - r0 < BB ? n - r0 : BB);
      stage_c<double>(L0, F + r0 + k * n, n, rv, kb);  // (r, kx) at L0[kx * LDS_ + r]
      double bv[16], cn[2][2][4];
      auto prefetch = [&](int64_t c) {
        const int cv = int(n - c < BB ? n - c : BB);
        const double RBT_AS_GLOBAL *pb = Fd + k + (c + (bcol < cv ? bcol : 0)) * n;
        const int rl = kb - 1;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const double x = pb[bseg + e < kb ? bseg + e : rl];
          bv[e] = (bcol < cv && bseg + e < kb) ? x : 0.0;
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const int col = wn * 32 + 16 * j + l16;
            const int cc = col < cv ? col : cv - 1;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = wm * 32 + 16 * i + lk + 4 * v;
              const double x = Fd[(r0 + (row < rv ? row : rv - 1)) + (c + cc) * n];
              cn[i][j][v] = (row < rv && col < cv) ? x : 0.0;
            }
          }
      };
      prefetch(k + kb);
      for (int64_t c0 = k + kb; c0 < n; c0 += BB) {
        const int cv = int(n - c0 < BB ? n - c0 : BB);
#pragma unroll
        for (int e = 0; e < 16; ++e) L1d[bcol * LDS_ + bseg + e] = bv[e];  // (kx, nx) at L1[nx * LDS_ + kx]
        double cc[2][2][4];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) cc[i][j][v] = cn[i][j][v];
        __syncthreads();
        if (c0 + BB < n) prefetch(c0 + BB);
        tile_mma_c<double>([&](int m, int kx) { return L0d[kx * LDS_ + m]; },
                           [&](int kx, int nx) { return L1d[nx * LDS_ + kx]; }, acc64);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const int col = wn * 32 + 16 * j + l16;
            if (col >= cv) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = wm * 32 + 16 * i + lk + 4 * v;
              if (row < rv) Fd[(r0 + row) + (c0 + col) * n] = cc[i][j][v] - acc64[i][j][v];
            }
          }
        __syncthreads();
      }
    }
    __syncthreads();
  }
}

// One-sided transform of the n x nrhs block Y (ld ldy) with coefficients C,
// in passes of at most three layers (op T: layers d..1, op N: 1..d).
template <int OP>
__device__ __noinline__ void transform_vec_sys(const Sys &s, int d, double *Y, int64_t ldy_in,
                                               const double *C) {
  if (d == 0) return;
  double RBT_AS_GLOBAL *Yg = (double RBT_AS_GLOBAL *)wave_uniform(Y);
  const double RBT_AS_GLOBAL *Cg = (const double RBT_AS_GLOBAL *)wave_uniform(C);
  const int64_t ldy = wave_uniform(ldy_in), n = wave_uniform(s.n), q = wave_uniform(s.q);
  const int nrhs = int(wave_uniform(s.nrhs));
  for (int k = 0; k < (d + 2) / 3; ++k) {
    // op T: passes (d-2..d), (d-5..d-3), ...; op N: (1..3), (4..6), ...
    const int hi = OP == RBT_OP_T ? d - 3 * k : (3 * k + 3 < d ? 3 * k + 3 : d);
    const int lo = OP == RBT_OP_T ? (hi - 2 > 1 ? hi - 2 : 1) : 3 * k + 1;
    const dev::Pass ps = dev::make_pass(n, q, d, lo, hi, s.rot, s.sides);
    const int ng = int(ps.ngroups);
    for (int e = threadIdx.x; e < ng * nrhs; e += BT) {
      const int gr = e % ng, j = e / ng;
      const int64_t rb = dev::group_base(ps, gr);
      if (rb >= n) continue;
      switch (hi - lo + 1) {
        case 1: dev::transform_vec_block<1, OP>(Yg, ldy, j, Cg, ps, rb); break;
        case 2: dev::transform_vec_block<2, OP>(Yg, ldy, j, Cg, ps, rb); break;
        default: dev::transform_vec_block<3, OP>(Yg, ldy, j, Cg, ps, rb); break;
      }
    }
    __syncthreads();
  }
}

// Y (n x nrhs FP64 storage, ld ldy) <- (L U)^-1 Y (LOWER: L, else U) with
// the factors and the inverses of their diagonal blocks, in the factors'
// arithmetic type TF (FP32 for the low-precision pass: a value of Y is
// rounded to FP32 when the sweep first reads it and every update is an FP32
// operation; FP64 for the fallback), right-looking: for each diagonal block
// b in sweep order, x_b = Dinv_b y_b (threads: 64 rows x 4 segments of 16,
// reduced in LDS), then every row still to be solved takes
// y_m -= F[m, block b] x_b as a matrix-core product of 16-row tiles of the
// factor (16 loads per lane, issued one tile ahead) with x_b (16 values per
// lane, held in registers for the step). Operand and output layout: mma16.h.
// NRT: right-hand sides of the inverse product (>= N).
template <bool LOWER, int NRT, typename TF>
__device__ __noinline__ void sweep(const Sys &s, double *Y_in, int64_t ldy_in, double *L0) {
  typedef Mma16<TF> M;
  typedef typename Lds<TF>::T lds_t;
  const TF RBT_AS_GLOBAL *F = (const TF RBT_AS_GLOBAL *)fmat<TF>(s);
  const TF RBT_AS_GLOBAL *Inv = (const TF RBT_AS_GLOBAL *)wave_uniform(s.Inv);
  double RBT_AS_GLOBAL *Y = (double RBT_AS_GLOBAL *)wave_uniform(Y_in);
  const int64_t ldy = wave_uniform(ldy_in);
  const int64_t n = wave_uniform(s.n);
  const int N = int(wave_uniform(s.nrhs));
  const int tid = threadIdx.x, i = tid & 63, sg = tid >> 6;
  const int lane = tid & 63, wave = tid >> 6, l16 = lane & 15, lk = lane >> 4;
  lds_t *Ll = (lds_t *)L0;
  TF RBT_AS_LDS(*part)[BB][NRT] = reinterpret_cast<TF RBT_AS_LDS(*)[BB][NRT]>(Ll);  // [4][64][NRT]
  TF RBT_AS_LDS(*xs)[NR] = reinterpret_cast<TF RBT_AS_LDS(*)[NR]>(Ll + 4 * BB * NRT);  // [64][16]
  // FP32 refinement step: y_b and the first x_b
  TF RBT_AS_LDS(*ys)[NR] = reinterpret_cast<TF RBT_AS_LDS(*)[NR]>(Ll + 4 * BB * NRT + BB * NR);
  TF RBT_AS_LDS(*x0s)[NR] = reinterpret_cast<TF RBT_AS_LDS(*)[NR]>(Ll + 4 * BB * NRT + 2 * BB * NR);
  const int64_t nblk = (n + BB - 1) / BB;
  for (int64_t t = 0; t < nblk; ++t) {
    const int64_t b = LOWER ? t : nblk - 1 - t;
    const int64_t r0 = b * BB;
    const int kb = int(n - r0 < BB ? n - r0 : BB);
    // y_b -> LDS
    if (sg == 0) {
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        const TF y = (i < kb && c < N) ? TF(Y[(r0 + i) + int64_t(c) * ldy]) : TF(0);
        xs[i][c] = y;
        if constexpr (sizeof(TF) == 4) ys[i][c] = y;
      }
    }
    __syncthreads();
    // x_b = Dinv y_b: part[sg][i][:] = sum over this segment's 16 columns of
    // Dinv(i, kx) xs[kx][:], then the four segments are added
    const TF RBT_AS_GLOBAL *Db = Inv + b * BB * BB;
    // (entries read from the inverse where they are used: an array of them
    // held through the loops below would be indexed dynamically)
    auto dinv = [&](int q) {
      const int kx = sg * 16 + q;
      const TF d = Db[i + kx * BB];
      return LOWER ? (i > kx ? d : (i == kx ? TF(1) : TF(0))) : (i <= kx ? d : TF(0));
    };
    auto part_sum = [&](int c) {
      return (part[0][i][c] + part[1][i][c]) + (part[2][i][c] + part[3][i][c]);
    };
    {
      TF acc[NRT];
#pragma unroll
      for (int c = 0; c < NRT; ++c) acc[c] = TF(0);
#pragma unroll 2
      for (int q = 0; q < 16; ++q) {
        const TF v = dinv(q);
#pragma unroll
        for (int c = 0; c < NRT; ++c) acc[c] += v * xs[sg * 16 + q][c];
      }
#pragma unroll
      for (int c = 0; c < NRT; ++c) part[sg][i][c] = acc[c];
    }
    __syncthreads();
    if (sg == 0) {
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        TF x = TF(0);
        if (c < NRT && i < kb && c < N) x = part_sum(c < NRT ? c : 0);
        xs[i][c] = x;
        if constexpr (sizeof(TF) == 4)
          x0s[i][c] = x;
        else if (i < kb && c < N)
          Y[(r0 + i) + int64_t(c) * ldy] = double(x);
      }
    }
    __syncthreads();
    if constexpr (sizeof(TF) == 4) {
      // FP32: one refinement step against the diagonal block itself, so the
      // block solve is not limited to kappa(block) u32 (the product with an
      // explicit inverse alone is): r = y_b - D x_b, x_b += Dinv r
      {
        const int ic = i < kb ? i : kb - 1;
        TF acc[NRT];
#pragma unroll
        for (int c = 0; c < NRT; ++c) acc[c] = TF(0);
#pragma unroll 2
        for (int q = 0; q < 16; ++q) {
          const int kx = sg * 16 + q;
          const TF f = F[(r0 + ic) + (r0 + (kx < kb ? kx : kb - 1)) * n];
          const bool in = i < kb && kx < kb;
          const TF v = LOWER ? (i == kx ? TF(1) : (in && kx < i ? f : TF(0)))
                             : (in && kx >= i ? f : (i == kx ? TF(1) : TF(0)));
#pragma unroll
          for (int c = 0; c < NRT; ++c) acc[c] += v * xs[kx][c];
        }
#pragma unroll
        for (int c = 0; c < NRT; ++c) part[sg][i][c] = acc[c];
      }
      __syncthreads();
      if (sg == 0) {
#pragma unroll
        for (int c = 0; c < NR; ++c)
          xs[i][c] = (c < NRT && i < kb && c < N) ? ys[i][c] - part_sum(c < NRT ? c : 0) : TF(0);
      }
      __syncthreads();
      {
        TF acc[NRT];
#pragma unroll
        for (int c = 0; c < NRT; ++c) acc[c] = TF(0);
#pragma unroll 2
        for (int q = 0; q < 16; ++q) {
          const TF v = dinv(q);
#pragma unroll
          for (int c = 0; c < NRT; ++c) acc[c] += v * xs[sg * 16 + q][c];
        }
#pragma unroll
        for (int c = 0; c < NRT; ++c) part[sg][i][c] = acc[c];
      }
      __syncthreads();
      if (sg == 0) {
#pragma unroll
        for (int c = 0; c < NR; ++c) {
          TF x = x0s[i][c];
          if (c < NRT && i < kb && c < N) x += part_sum(c < NRT ? c : 0);
          xs[i][c] = x;
          if (i < kb && c < N) Y[(r0 + i) + int64_t(c) * ldy] = double(x);
        }
      }
      __syncthreads();
    }
    // rows still to be solved: after the block (L) or before it (U)
    const int64_t lo = LOWER ? r0 + kb : 0, hi = LOWER ? n : r0;
    if (hi > lo) {
      TF xb[16];
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) xb[kk] = xs[lk + 4 * kk][l16];
      const int64_t ntile = (hi - lo + 15) / 16;
      auto load_tile = [&](int64_t tt, TF (&av)[16]) {
        const int64_t m = lo + 16 * tt + l16;
        const int64_t mc = m < hi ? m : hi - 1;
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
          const int kx = lk + 4 * kk;
          av[kk] = F[mc + (r0 + (kx < kb ? kx : kb - 1)) * n];
        }
      };
      // the lane's four entries of Y in the tile (column l16), read with the
      // tile's factor entries one tile ahead: a row always belongs to the
      // same wavefront (lo moves by whole 4-tile rounds), so no other
      // wavefront writes them in between
      const int yc = l16 < N ? l16 : N - 1;
      auto load_y = [&](int64_t tt, double (&yv)[4]) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t m = lo + 16 * tt + M::row(lk, v);
          yv[v] = Y[(m < hi ? m : hi - 1) + int64_t(yc) * ldy];
        }
      };
      TF av[16], an[16];
      double yv[4], yn[4];
      int64_t tt = wave;
      if (tt < ntile) {
        load_tile(tt, av);
        load_y(tt, yv);
      }
      for (; tt < ntile; tt += 4) {
        if (tt + 4 < ntile) {
          load_tile(tt + 4, an);
          load_y(tt + 4, yn);
        }
        typename M::v4 o = {TF(0), TF(0), TF(0), TF(0)};
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
          const TF a = (lk + 4 * kk < kb && lo + 16 * tt + l16 < hi) ? av[kk] : TF(0);
          o = M::mma(a, xb[kk], o);
        }
        if (l16 < N) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t m = lo + 16 * tt + M::row(lk, v);
            if (m < hi) Y[m + int64_t(l16) * ldy] = double(TF(yv[v]) - o[v]);
          }
        }
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) av[kk] = an[kk];
#pragma unroll
        for (int v = 0; v < 4; ++v) yv[v] = yn[v];
      }
    }
    __syncthreads();
  }
}

// R = B - A X (FP64, original A), Eq. 7 backward error (max over columns);
// with_anorm: also ||A||_inf into *anorm. One pass over A (rows on
// threads, X staged in LDS by chunks of columns), then the column maxima of
// |R|, |X|, |B| in a second, small pass.
template <int NRT>
__device__ __noinline__ double residual(const Sys &s, double *L0, bool with_anorm, double *anorm) {
  const int64_t n = wave_uniform(s.n);
  const int N = int(wave_uniform(s.nrhs));
  const int64_t lda = wave_uniform(s.lda), ldx = wave_uniform(s.ldx), ldb = wave_uniform(s.ldb);
  const int tid = threadIdx.x;
  constexpr int KC = 256;  // columns of A per staged chunk of X
  ldouble *Ll = (ldouble *)L0;
  double RBT_AS_LDS(*xs)[NRT] = reinterpret_cast<double RBT_AS_LDS(*)[NRT]>(Ll);  // [KC][NRT]
  double *red = L0 + KC * NR;  // (wg_nanmax takes a plain pointer)
  const double RBT_AS_GLOBAL *Ag = (const double RBT_AS_GLOBAL *)wave_uniform(s.A);
  const double RBT_AS_GLOBAL *Xg = (const double RBT_AS_GLOBAL *)wave_uniform(s.Xm);
  const double RBT_AS_GLOBAL *Bg = (const double RBT_AS_GLOBAL *)wave_uniform(s.Bm);
  double RBT_AS_GLOBAL *Rg = (double RBT_AS_GLOBAL *)wave_uniform(s.R);
  double amax = 0.0;
  for (int64_t m0 = 0; m0 < n; m0 += BT) {
    const int64_t m = m0 + tid;
    double acc[NRT];
#pragma unroll
    for (int c = 0; c < NRT; ++c) acc[c] = 0.0;
    double asum = 0.0;
    for (int64_t k0 = 0; k0 < n; k0 += KC) {
      const int kc = int(n - k0 < KC ? n - k0 : KC);
      __syncthreads();
      for (int e = tid; e < KC * NRT; e += BT) {
        const int kx = e % KC, c = e / KC;  // consecutive threads: consecutive rows of X
        xs[kx][c] = (kx < kc && c < N) ? Xg[(k0 + kx) + int64_t(c) * ldx] : 0.0;
      }
      __syncthreads();
      if (m < n) {
        const double RBT_AS_GLOBAL *Ap = Ag + m + k0 * lda;
        // batches of 32 loads in flight (kc is a multiple of 32 except at the
        // end): all issued before the first product uses one
        int kx = 0;
#pragma unroll 1
        for (; kx + 32 <= kc; kx += 32) {
          double av[32];
          const double RBT_AS_GLOBAL *p = Ap + int64_t(kx) * lda;
#pragma unroll
          for (int q = 0; q < 32; ++q) av[q] = p[int64_t(q) * lda];
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int q = 0; q < 32; ++q) {
            if (with_anorm) asum += fabs(av[q]);
#pragma unroll
            for (int c = 0; c < NRT; ++c) acc[c] += av[q] * xs[kx + q][c];
          }
        }
#pragma unroll 1
        for (; kx < kc; ++kx) {
          const double a = Ap[int64_t(kx) * lda];
          if (with_anorm) asum += fabs(a);
#pragma unroll
          for (int c = 0; c < NRT; ++c) acc[c] += a * xs[kx][c];
        }
      }
    }
    if (m < n) {
      amax = nanmax(amax, asum);
#pragma unroll
      for (int c = 0; c < NRT; ++c)
        if (c < N) Rg[m + int64_t(c) * n] = Bg[m + int64_t(c) * ldb] - acc[c];
    }
  }
  __syncthreads();
  if (with_anorm) {
    const double an = wg_nanmax(amax, red);
    if (tid == 0) *anorm = an;
    __syncthreads();
  }
  const double an = *anorm;
  double be = 0.0;
  for (int c = 0; c < N; ++c) {
    double rm = 0.0, xm = 0.0, bm = 0.0;
    for (int64_t m = tid; m < n; m += BT) {
      rm = nanmax(rm, fabs(Rg[m + int64_t(c) * n]));
      xm = nanmax(xm, fabs(Xg[m + int64_t(c) * ldx]));
      bm = nanmax(bm, fabs(Bg[m + int64_t(c) * ldb]));
    }
    const double r = wg_nanmax(rm, red);
    const double x = wg_nanmax(xm, red);
    const double b = wg_nanmax(bm, red);
    const double den = an * x + b;
    const double e = den > 0.0 ? r / den : (r > 0.0 ? INFINITY : (r != r ? r : 0.0));
    be = nanmax(be, e);
  }
  return be;
}

// X = V (LU)^-1 U^T B with the factors of storage type TF, then classical
// refinement in FP64 until the Eq. 7 backward error is <= tol, max_iter
// corrections, stagnation or NaN.
// project: when a fallback follows (the low-precision pass with FP64 factors
// available), also stop once the observed rate of the last correction,
// extrapolated, cannot reach tol within max_iter steps (the batch's slowest
// systems are the large ones whose refinement fails; their hopeless steps
// are spent before the fallback's elimination).
template <int NRT, typename TF>
__device__ void refine_system(const Sys &s, int d, double tol, int max_iter, double *L0,
                              double *anorm_sh, int *it_out, double *be_out, bool project) {
  const int64_t n = s.n;
  double RBT_AS_GLOBAL *Xg = (double RBT_AS_GLOBAL *)s.Xm;
  const double RBT_AS_GLOBAL *Bg = (const double RBT_AS_GLOBAL *)s.Bm;
  const double RBT_AS_GLOBAL *Rg = (const double RBT_AS_GLOBAL *)s.R;
  for (int64_t e = threadIdx.x; e < n * s.nrhs; e += BT)
    Xg[(e % n) + (e / n) * s.ldx] = Bg[(e % n) + (e / n) * s.ldb];
  __syncthreads();
  transform_vec_sys<RBT_OP_T>(s, d, s.Xm, s.ldx, s.U);
  sweep<true, NRT, TF>(s, s.Xm, s.ldx, L0);
  sweep<false, NRT, TF>(s, s.Xm, s.ldx, L0);
  if (s.sides != 1) transform_vec_sys<RBT_OP_N>(s, d, s.Xm, s.ldx, s.V);  // x = V x~
  int it = 0, stalled = 0;
  double be = 0.0, best = INFINITY;
  for (;;) {
    be = residual<NRT>(s, L0, it == 0, anorm_sh);
    if (be <= tol || it >= max_iter) break;  // a NaN error never looks converged
    // stagnation: two corrections in a row that do not improve the best
    // backward error by 10 % end the refinement (reported not converged)
    stalled = (be < 0.9 * best) ? 0 : stalled + 1;
    if (project && it >= 1 && be < best) {
      // steps still needed at rate be / best: log(tol / be) / log(be / best)
      const double need = log(tol / be) / log(be / best);
      if (double(it) + need > double(max_iter)) break;
    }
    if (be < best) best = be;
    if (stalled >= 2 || be != be) break;
    transform_vec_sys<RBT_OP_T>(s, d, s.R, n, s.U);
    sweep<true, NRT, TF>(s, s.R, n, L0);
    sweep<false, NRT, TF>(s, s.R, n, L0);
    if (s.sides != 1) transform_vec_sys<RBT_OP_N>(s, d, s.R, n, s.V);
    for (int64_t e = threadIdx.x; e < n * s.nrhs; e += BT)
      Xg[(e % n) + (e / n) * s.ldx] += Rg[e];
    __syncthreads();
    ++it;
  }
  *it_out = it;
  *be_out = be;
}

// A~ = U^T A V into the factor storage of type TF (FP32 for the
// low-precision pass, FP64 for the fallback), in passes of at most three
// layers from layer d down: the first reads A, the later ones the factor
// storage in place (each block of a pass belongs to one thread).
template <typename TF>
__device__ __noinline__ void transform_into(const Sys &s, int d) {
  const double RBT_AS_GLOBAL *Ag = (const double RBT_AS_GLOBAL *)wave_uniform(s.A);
  const double RBT_AS_GLOBAL *Ug = (const double RBT_AS_GLOBAL *)wave_uniform(s.U);
  const double RBT_AS_GLOBAL *Vg = (const double RBT_AS_GLOBAL *)wave_uniform(s.V);
  TF RBT_AS_GLOBAL *Fg = (TF RBT_AS_GLOBAL *)fmat<TF>(s);
  const int64_t n = wave_uniform(s.n), lda = wave_uniform(s.lda), q = wave_uniform(s.q);
  for (int hi = d, first = 1; first || hi >= 1; first = 0) {
    const int lo = d == 0 ? 1 : (hi - 2 > 1 ? hi - 2 : 1);
    const dev::Pass ps =
        d > 0 ? dev::make_pass(n, q, d, lo, hi, s.rot, s.sides) : dev::identity_pass(n);
    const int P = d > 0 ? hi - lo + 1 : 0;
    for (int64_t e = threadIdx.x; e < ps.ngroups * ps.ngroups; e += BT) {
      const int64_t gr = e % ps.ngroups, gc = e / ps.ngroups;
      const int64_t rb = dev::group_base(ps, gr), cb = dev::group_base(ps, gc);
      if (rb >= n || cb >= n) continue;
      if (first) {
        switch (P) {
          case 0: dev::transform2_block<0, TF>(Ag, lda, Fg, n, Ug, Vg, ps, rb, cb); break;
          case 1: dev::transform2_block<1, TF>(Ag, lda, Fg, n, Ug, Vg, ps, rb, cb); break;
          case 2: dev::transform2_block<2, TF>(Ag, lda, Fg, n, Ug, Vg, ps, rb, cb); break;
          default: dev::transform2_block<3, TF>(Ag, lda, Fg, n, Ug, Vg, ps, rb, cb); break;
        }
      } else {
        switch (P) {
          case 1: dev::transform2_block<1, TF>(Fg, n, Fg, n, Ug, Vg, ps, rb, cb); break;
          case 2: dev::transform2_block<2, TF>(Fg, n, Fg, n, Ug, Vg, ps, rb, cb); break;
          default: dev::transform2_block<3, TF>(Fg, n, Fg, n, Ug, Vg, ps, rb, cb); break;
        }
      }
    }
    __syncthreads();
    if (d == 0) break;
    hi = lo - 1;
  }
}

template <bool BF16U>
__device__ void solve_system(const Args &a, const BatchDesc &D, float *fbase, double *dbase,
                             double *f64base, double *L0, double *L1, int *info_sh,
                             double *anorm_sh) {
  const int tid = threadIdx.x;
  const int d = a.depth;
  Sys s;
  s.n = D.n;
  s.nrhs = D.nrhs;
  {  // m = 2^d g ceil(n / (2^d g)), q = m / 2^d
    const int64_t g = (int64_t(1) << d) * a.granule;
    s.q = d > 0 ? (((s.n + g - 1) / g) * g) >> d : s.n;
  }
  s.rot = a.kind == 1 ? 1 : 0;
  s.sides = a.sides;
  s.F = fbase + D.f_off;
  s.F64 = f64base ? f64base + D.f64_off : nullptr;
  s.U = dbase + D.d_off;
  s.V = s.U + s.n * d;
  s.Inv = s.V + s.n * d;
  s.R = s.Inv + ((s.n + BB - 1) / BB) * BB * BB;
  s.A = a.A[D.sys];
  s.lda = a.lda[D.sys];
  s.Bm = a.B[D.sys];
  s.ldb = a.ldb[D.sys];
  s.Xm = a.X[D.sys];
  s.ldx = a.ldx[D.sys];
  const int64_t n = s.n;
  const uint64_t seed = dev::splitmix_at(a.seed, uint64_t(D.sys));
  if (tid == 0) *info_sh = 0;
  // coefficients
  for (int64_t e = tid; e < 2 * n * d; e += BT) {
    const int side = e >= n * d ? 1 : 0;
    const int64_t rem = e - side * n * d;
    s.U[e] = s.rot ? dev::rotation_coefficient(seed, rem % n, side, int(rem / n) + 1, n, s.q, d)
                   : dev::coefficient(seed, rem % n, side, int(rem / n) + 1);
  }
  __syncthreads();
  const double tol = a.tol < 0.0 ? -a.tol * double(n) * 0x1.0p-52 : a.tol;
  int it = 0, path = 0;
  double be = 0.0;
  // low precision first; if its refinement fails, FP64 factors (fallback)
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      if (be <= tol || s.F64 == nullptr) break;
      path = 1;
      if (tid == 0) *info_sh = 0;
      __syncthreads();
    }
    if (pass == 0)
      transform_into<float>(s, d);
    else
      transform_into<double>(s, d);
    if (pass == 0 && s.n >= a.ct2_min_n)
      eliminate<float, BF16U, 2>(s, L0, L1, info_sh);
    else if (pass == 0)
      eliminate<float, BF16U, 1>(s, L0, L1, info_sh);
    else
      eliminate<double, false>(s, L0, L1, info_sh);
    int it_p = 0;
    if (pass == 0) {
      if (s.nrhs <= 1)
        refine_system<1, float>(s, d, tol, a.max_iter, L0, anorm_sh, &it_p, &be, s.F64 != nullptr);
      else if (s.nrhs <= 4)
        refine_system<4, float>(s, d, tol, a.max_iter, L0, anorm_sh, &it_p, &be, s.F64 != nullptr);
      else
        refine_system<NR, float>(s, d, tol, a.max_iter, L0, anorm_sh, &it_p, &be, s.F64 != nullptr);
    } else {
      if (s.nrhs <= 1)
        refine_system<1, double>(s, d, tol, a.max_iter, L0, anorm_sh, &it_p, &be, false);
      else if (s.nrhs <= 4)
        refine_system<4, double>(s, d, tol, a.max_iter, L0, anorm_sh, &it_p, &be, false);
      else
        refine_system<NR, double>(s, d, tol, a.max_iter, L0, anorm_sh, &it_p, &be, false);
    }
    it += it_p;
  }
  if (tid == 0 && a.path) a.path[D.sys] = path;
  if (tid == 0) {
    if (a.iters) a.iters[D.sys] = it;
    if (a.berr) a.berr[D.sys] = be;
    if (a.info) a.info[D.sys] = *info_sh;
  }
  __syncthreads();
}

template <bool BF16U>
__global__ void __launch_bounds__(BT, 2) k_batched(Args a) {
  __shared__ __attribute__((aligned(16))) double lds[kR0Doubles + kR1Doubles];
  double *L0 = lds, *L1 = lds + kR0Doubles;
  __shared__ int64_t tk_sh;
  __shared__ int info_sh;
  __shared__ double anorm_sh;
  BatchHeader *hdr = reinterpret_cast<BatchHeader *>(a.work);
  // a plan for other sizes, depth or precision, or a workspace too small for
  // it: no system is solved, and every system reports it (info -1, berr NaN,
  // path -1), so no caller mistakes the untouched X for a solution
  if (hdr->batch != a.batch || hdr->depth != a.depth || hdr->prec != a.prec ||
      hdr->total_bytes < 0 || size_t(hdr->total_bytes) > a.work_bytes) {
    for (int64_t sys = int64_t(blockIdx.x) * BT + threadIdx.x; sys < a.batch;
         sys += int64_t(gridDim.x) * BT) {
      if (a.path) a.path[sys] = -1;
      if (a.iters) a.iters[sys] = 0;
      if (a.berr) a.berr[sys] = __builtin_nan("");
      if (a.info) a.info[sys] = -1;
    }
    return;
  }
  const BatchDesc *desc = reinterpret_cast<const BatchDesc *>(a.work + kBatchTableOffset);
  float *fbase = reinterpret_cast<float *>(a.work + hdr->f_off_bytes);
  double *dbase = reinterpret_cast<double *>(a.work + hdr->d_off_bytes);
  double *f64base =
      hdr->f64_off_bytes > 0 ? reinterpret_cast<double *>(a.work + hdr->f64_off_bytes) : nullptr;
  // Each round takes one ticket; every ticket below `batch` is taken once
  // over the grid, so no workgroup needs more than batch + 1 rounds. The
  // bound makes the loop's end independent of the ticket word's value.
  for (int64_t round = 0; round <= a.batch; ++round) {
    if (threadIdx.x == 0) tk_sh = atomicAdd(&hdr->ticket, 1);
    __syncthreads();
    const int64_t t = wave_uniform(tk_sh);
    __syncthreads();
    if (t < 0 || t >= a.batch) break;
    const BatchDesc D = desc[t];
    // systems without work (n = 0, or no right-hand side) are not solved;
    // the plan queues them last
    if (D.n > 0 && D.nrhs > 0) {
      solve_system<BF16U>(a, D, fbase, dbase, f64base, L0, L1, &info_sh, &anorm_sh);
    } else if (threadIdx.x == 0) {
      if (a.path) a.path[D.sys] = 0;
      if (a.iters) a.iters[D.sys] = 0;
      if (a.berr) a.berr[D.sys] = 0.0;
      if (a.info) a.info[D.sys] = 0;
    }
  }
}

__global__ void k_reset_ticket(void *work) {
  if (threadIdx.x == 0) reinterpret_cast<BatchHeader *>(work)->ticket = 0;
}

}  // namespace

hipError_t launch_batched(int64_t batch, void *work, size_t work_bytes, const double *const *A,
                          const int64_t *lda, const double *const *B, const int64_t *ldb,
                          double *const *X, const int64_t *ldx, int depth, uint64_t seed,
                          int prec, double tol, int max_iter, int32_t *iters, double *berr,
                          int32_t *info, int32_t *path, int grid, int64_t ct2_min_n,
                          hipStream_t s) {
  if (ct2_min_n < 0) return hipErrorInvalidValue;
  Args a;
  a.batch = batch;
  a.work = static_cast<char *>(work);
  a.work_bytes = work_bytes;
  a.A = A;
  a.lda = lda;
  a.B = B;
  a.ldb = ldb;
  a.X = X;
  a.ldx = ldx;
  a.iters = iters;
  a.berr = berr;
  a.info = info;
  a.path = path;
  a.seed = seed;
  a.tol = tol;
  a.depth = depth;
  a.prec = prec;
  a.max_iter = max_iter;
  a.granule = butterfly_granule();
  a.kind = butterfly_kind();
  a.sides = butterfly_sides();
  a.ct2_min_n = ct2_min_n;
  hipLaunchKernelGGL(k_reset_ticket, dim3(1), dim3(64), 0, s, work);
  const dim3 g{unsigned(grid)}, b{unsigned(BT)};
  if (prec == RBT_BF16)
    hipLaunchKernelGGL((k_batched<true>), g, b, 0, s, a);
  else
    hipLaunchKernelGGL((k_batched<false>), g, b, 0, s, a);
  return hipGetLastError();
}

}  // namespace rbt
