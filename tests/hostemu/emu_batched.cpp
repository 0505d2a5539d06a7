// Host build of the batched solver for tests: the library's kernel source
// (k_batched.hip) and host plan (batch_plan.cpp) compiled as host C++ with
// the emulation header, driven from a file. Every buffer is its own heap
// allocation, and in the workspace only the header, the descriptor table
// and each system's areas are addressable: under AddressSanitizer any other
// access is reported.
//
//   emu_batched IN OUT
// IN (little-endian): int64 batch, depth, prec, max_iter, ct2_min_n, grid,
//   granule, kind, sides; uint64 seed; double tol; int64 n[batch],
//   nrhs[batch]; per system A (n x n, column-major) then B (n x nrhs).
// OUT: per system X (n x nrhs); int32 iters[batch]; double berr[batch];
//   int32 info[batch]; int32 path[batch]; uint64 divergent barriers; int64
//   final ticket word; uint64 1 if the header (but the ticket) and the
//   descriptor table are as planned, else 0.
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "internal.h"

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#include <sanitizer/asan_interface.h>
#define EMU_POISON(p, n) ASAN_POISON_MEMORY_REGION(p, n)
#define EMU_UNPOISON(p, n) ASAN_UNPOISON_MEMORY_REGION(p, n)
#endif
#endif
#ifndef EMU_POISON
#define EMU_POISON(p, n) ((void)(p), (void)(n))
#define EMU_UNPOISON(p, n) ((void)(p), (void)(n))
#endif

namespace {
int64_t g_granule = 1;
int g_kind = 0, g_sides = 2;
}  // namespace

namespace rbt {
// The library's structure options, fixed per run here.
int64_t butterfly_granule() { return g_granule; }
int butterfly_kind() { return g_kind; }
int butterfly_sides() { return g_sides; }
}  // namespace rbt

extern "C" unsigned long long emu_divergent_barriers();

namespace {

template <typename T>
void rd(FILE *f, T *p, size_t n) {
  if (n && std::fread(p, sizeof(T), n, f) != n) {
    std::fprintf(stderr, "emu_batched: short input\n");
    std::exit(2);
  }
}
template <typename T>
void wr(FILE *f, const T *p, size_t n) {
  if (n) std::fwrite(p, sizeof(T), n, f);
}

}  // namespace

int main(int argc, char **argv) {
  if (argc != 3) {
    std::fprintf(stderr, "usage: emu_batched IN OUT\n");
    return 2;
  }
  FILE *in = std::fopen(argv[1], "rb");
  if (!in) return 2;
  int64_t hdr[9];
  rd(in, hdr, 9);
  const int64_t batch = hdr[0], ct2_min_n = hdr[4];
  const int depth = int(hdr[1]), prec = int(hdr[2]), max_iter = int(hdr[3]), grid = int(hdr[5]);
  g_granule = hdr[6];
  g_kind = int(hdr[7]);
  g_sides = int(hdr[8]);
  uint64_t seed;
  double tol;
  rd(in, &seed, 1);
  rd(in, &tol, 1);
  std::vector<int64_t> n(batch), k(batch);
  rd(in, n.data(), batch);
  rd(in, k.data(), batch);
  std::vector<double *> A(batch), B(batch), X(batch);
  std::vector<int64_t> lda(batch), ldb(batch), ldx(batch);
  for (int64_t s = 0; s < batch; ++s) {
    const size_t na = size_t(n[s] * n[s]), nb = size_t(n[s] * k[s]);
    A[s] = static_cast<double *>(std::malloc(na * 8 + 1));
    B[s] = static_cast<double *>(std::malloc(nb * 8 + 1));
    X[s] = static_cast<double *>(std::malloc(nb * 8 + 1));
    rd(in, A[s], na);
    rd(in, B[s], nb);
    for (size_t e = 0; e < nb; ++e) X[s][e] = 0.0;
    lda[s] = ldb[s] = ldx[s] = n[s] > 0 ? n[s] : 1;
  }
  std::fclose(in);

  int rc = rbt::check_batch_sizes(batch, n.data(), k.data());
  if (rc) {
    std::fprintf(stderr, "emu_batched: sizes rejected (%d)\n", rc);
    return 2;
  }
  std::vector<rbt::BatchDesc> desc;
  const rbt::BatchPlanSizes z = rbt::batch_plan_sizes(batch, n.data(), k.data(), depth, &desc);
  const std::vector<char> image = rbt::batch_plan_image(batch, depth, prec, z, desc);
  char *work = static_cast<char *>(std::malloc(z.total));
  std::memcpy(work, image.data(), image.size());
  // only the header, the table and each system's areas are addressable
  EMU_POISON(work, z.total);
  EMU_UNPOISON(work, sizeof(rbt::BatchHeader));
  EMU_UNPOISON(work + rbt::kBatchTableOffset, size_t(batch) * sizeof(rbt::BatchDesc));
  for (const rbt::BatchDesc &D : desc) {
    EMU_UNPOISON(work + z.f_off + size_t(D.f_off) * 4, size_t(D.n * D.n) * 4);
    EMU_UNPOISON(work + z.d_off + size_t(D.d_off) * 8,
                 size_t(rbt::batched_sys_doubles(D.n, D.nrhs, depth)) * 8);
    EMU_UNPOISON(work + z.f64_off + size_t(D.f64_off) * 8, size_t(D.n * D.n) * 8);
  }
  std::vector<int32_t> iters(batch, -7), info(batch, -7), path(batch, -7);
  std::vector<double> berr(batch, -7.0);
  const hipError_t e = rbt::launch_batched(
      batch, work, z.total, A.data(), lda.data(), const_cast<const double *const *>(B.data()),
      ldb.data(), X.data(), ldx.data(), depth, seed, prec, tol, max_iter, iters.data(), berr.data(),
      info.data(), path.data(), grid, ct2_min_n, nullptr);
  if (e != hipSuccess) {
    std::fprintf(stderr, "emu_batched: launch rejected (%d)\n", int(e));
    return 2;
  }
  FILE *out = std::fopen(argv[2], "wb");
  if (!out) return 2;
  for (int64_t s = 0; s < batch; ++s) wr(out, X[s], size_t(n[s] * k[s]));
  wr(out, iters.data(), batch);
  wr(out, berr.data(), batch);
  wr(out, info.data(), batch);
  wr(out, path.data(), batch);
  const unsigned long long dv = emu_divergent_barriers();
  wr(out, &dv, 1);
  const int64_t ticket = reinterpret_cast<const rbt::BatchHeader *>(work)->ticket;
  wr(out, &ticket, 1);
  const size_t t0 = offsetof(rbt::BatchHeader, batch);
  const unsigned long long intact =
      std::memcmp(work + t0, image.data() + t0, sizeof(rbt::BatchHeader) - t0) == 0 &&
      std::memcmp(work + rbt::kBatchTableOffset, image.data() + rbt::kBatchTableOffset,
                  size_t(batch) * sizeof(rbt::BatchDesc)) == 0;
  wr(out, &intact, 1);
  std::fclose(out);
  EMU_UNPOISON(work, z.total);
  std::free(work);
  for (int64_t s = 0; s < batch; ++s) {
    std::free(A[s]);
    std::free(B[s]);
    std::free(X[s]);
  }
  return 0;
}
