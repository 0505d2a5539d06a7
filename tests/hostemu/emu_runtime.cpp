// Runtime of the host build of device code (tests only): workgroups run on a
// pool of host threads (EMU_THREADS, default 8), each taking the next
// workgroup index; the work-items of a workgroup are fibers on its thread
// (x86-64: a switch saves the callee-saved registers on the fiber's stack and
// swaps stack pointers, no system call), switched at barriers and wavefront
// operations. Reports,
// and aborts on: a deadlock (no fiber can run, some have not finished), a
// wavefront operation that lanes reach with different operations, and a
// workgroup that passes more than EMU_MAX_BARRIERS barriers (default 10^8;
// a loop that does not end). Barriers reached from different source lines
// by the work-items of one workgroup are counted (emu_divergent_barriers).
#include <sys/mman.h>

#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "hip/hip_runtime.h"

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#define EMU_ASAN 1
#include <sanitizer/common_interface_defs.h>
#endif
#endif

thread_local emu::Index threadIdx, blockIdx, blockDim, gridDim;

// emu_ctx_switch(from, to): save the callee-saved registers and the stack
// pointer in *from, continue on the stack `to` (System V x86-64 ABI).
extern "C" void emu_ctx_switch(void **from, void *to);
asm(R"(
  .text
  .globl emu_ctx_switch
  .type emu_ctx_switch,@function
emu_ctx_switch:
  pushq %rbp
  pushq %rbx
  pushq %r12
  pushq %r13
  pushq %r14
  pushq %r15
  movq %rsp, (%rdi)
  movq %rsi, %rsp
  popq %r15
  popq %r14
  popq %r13
  popq %r12
  popq %rbx
  popq %rbp
  ret
  .size emu_ctx_switch, .-emu_ctx_switch
)");

namespace emu {
namespace {

constexpr size_t kStack = size_t(1) << 20;
enum State { kReady, kBarrier, kWave, kDone };

struct Fiber {
  void *sp = nullptr;
  char *stack = nullptr;
  State state = kReady;
  uint64_t wait_gen = 0;
  const char *file = "";
  int line = 0;
  void *fake_stack = nullptr;
};

struct Wave {
  int live = 0, arrived = 0;
  uint64_t gen = 0;
  WaveFn fn = nullptr;
  int ctx = 0;
  alignas(64) unsigned char in[64][64];
  alignas(64) unsigned char out[64][64];
};

struct Block {
  std::vector<Fiber> f;
  std::vector<Wave> w;
  unsigned n = 0;
  int live = 0, arrived = 0;
  uint64_t gen = 0, barriers = 0;
  const char *bfile = nullptr;
  int bline = 0;
  void *sched_sp = nullptr;
  int cur = -1;
  const std::function<void()> *body = nullptr;
  const void *sched_bottom = nullptr;
  size_t sched_size = 0;
};

thread_local Block g_blk;
std::atomic<uint64_t> g_divergent{0};
uint64_t g_max_barriers = 100000000ull;

void fail(const char *what) {
  Block &B = g_blk;
  std::fprintf(stderr, "emu: %s (block %u, fiber %d)\n", what, blockIdx.x, B.cur);
  int shown = 0;
  for (unsigned i = 0; i < B.n && shown < 16; ++i) {
    const Fiber &F = B.f[i];
    if (F.state == kDone) continue;
    std::fprintf(stderr, "  item %u: %s, last barrier %s:%d\n", i,
                 F.state == kBarrier ? "at a barrier" : F.state == kWave ? "in a wavefront op" : "runnable",
                 F.file, F.line);
    ++shown;
  }
  std::fflush(stderr);
  std::abort();
}

void to_scheduler(int idx, bool exiting) {
  Block &B = g_blk;
  Fiber &F = B.f[idx];
#ifdef EMU_ASAN
  __sanitizer_start_switch_fiber(exiting ? nullptr : &F.fake_stack, B.sched_bottom, B.sched_size);
#endif
  emu_ctx_switch(&F.sp, B.sched_sp);
#ifdef EMU_ASAN
  __sanitizer_finish_switch_fiber(F.fake_stack, &B.sched_bottom, &B.sched_size);
#endif
  (void)exiting;
}

void complete_wave(Wave &W) {
  W.fn(W.in, W.out, W.ctx);
  W.arrived = 0;
  ++W.gen;
}

void complete_barrier() {
  Block &B = g_blk;
  B.arrived = 0;
  ++B.gen;
  if (++B.barriers > g_max_barriers) fail("barrier limit reached (a loop that does not end?)");
}

void fiber_main() {
  Block &B = g_blk;
  const int idx = B.cur;
#ifdef EMU_ASAN
  __sanitizer_finish_switch_fiber(nullptr, &B.sched_bottom, &B.sched_size);
#endif
  (*B.body)();
  Fiber &F = B.f[idx];
  F.state = kDone;
  --B.live;
  Wave &W = B.w[idx / 64];
  --W.live;
  if (W.arrived > 0 && W.arrived == W.live) complete_wave(W);
  if (B.arrived > 0 && B.arrived == B.live) complete_barrier();
  to_scheduler(idx, true);
  fail("finished fiber resumed");
}

void run_block(unsigned n, dim3 block) {
  Block &B = g_blk;
  if (B.f.size() < n) {
    const size_t old = B.f.size();
    B.f.resize(n);
    for (size_t i = old; i < n; ++i) {
      void *p = mmap(nullptr, kStack, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
      if (p == MAP_FAILED) fail("mmap of a fiber stack failed");
      B.f[i].stack = static_cast<char *>(p);
    }
  }
  B.n = n;
  B.live = int(n);
  B.arrived = 0;
  B.bfile = nullptr;
  B.w.assign((n + 63) / 64, Wave{});
  for (unsigned w = 0; w < B.w.size(); ++w) B.w[w].live = int(n - 64 * w < 64 ? n - 64 * w : 64);
  for (unsigned i = 0; i < n; ++i) {
    Fiber &F = B.f[i];
    F.state = kReady;
    F.file = "";
    F.line = 0;
    F.fake_stack = nullptr;
    // first switch in: six zero registers, then "return" into fiber_main
    // with the stack aligned as after a call
    void **top = reinterpret_cast<void **>(F.stack + kStack);
    top[-1] = nullptr;
    top[-2] = reinterpret_cast<void *>(&fiber_main);
    for (int r = 3; r <= 8; ++r) top[-r] = nullptr;
    F.sp = top - 8;
  }
  for (;;) {
    bool ran = false;
    unsigned done = 0;
    for (unsigned i = 0; i < n; ++i) {
      Fiber &F = B.f[i];
      if (F.state == kDone) {
        ++done;
        continue;
      }
      const bool ready = F.state == kReady || (F.state == kBarrier && B.gen != F.wait_gen) ||
                         (F.state == kWave && B.w[i / 64].gen != F.wait_gen);
      if (!ready) continue;
      F.state = kReady;
      threadIdx = Index{i % block.x, (i / block.x) % block.y, i / (block.x * block.y)};
      B.cur = int(i);
      void *fake = nullptr;
#ifdef EMU_ASAN
      __sanitizer_start_switch_fiber(&fake, F.stack, kStack);
#endif
      emu_ctx_switch(&B.sched_sp, F.sp);
#ifdef EMU_ASAN
      __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#endif
      (void)fake;
      ran = true;
    }
    if (done == n) break;
    if (!ran) fail("deadlock: no work-item can continue");
  }
  B.cur = -1;
}

}  // namespace

void sync_threads(const char *file, int line) {
  Block &B = g_blk;
  const int i = B.cur;
  Fiber &F = B.f[i];
  if (B.arrived == 0) {
    B.bfile = file;
    B.bline = line;
  } else if (line != B.bline || std::strcmp(file, B.bfile) != 0) {
    ++g_divergent;
  }
  F.file = file;
  F.line = line;
  if (++B.arrived == B.live) {
    complete_barrier();
    return;
  }
  F.state = kBarrier;
  F.wait_gen = B.gen;
  to_scheduler(i, false);
}

void wave_op(WaveFn fn, int ctx, const void *in, size_t nin, void *out, size_t nout) {
  Block &B = g_blk;
  const int i = B.cur;
  Wave &W = B.w[i / 64];
  const int lane = i % 64;
  if (W.arrived == 0) {
    W.fn = fn;
    W.ctx = ctx;
  } else if (W.fn != fn || W.ctx != ctx) {
    fail("lanes of one wavefront reached different wavefront operations");
  }
  std::memcpy(W.in[lane], in, nin);
  if (++W.arrived == W.live) {
    complete_wave(W);
  } else {
    Fiber &F = B.f[i];
    F.state = kWave;
    F.wait_gen = W.gen;
    to_scheduler(i, false);
  }
  std::memcpy(out, W.out[lane], nout);
}

void launch(dim3 grid, dim3 block, const std::function<void()> &body) {
  if (const char *e = std::getenv("EMU_MAX_BARRIERS")) g_max_barriers = std::strtoull(e, nullptr, 10);
  unsigned nthreads = 8;
  if (const char *e = std::getenv("EMU_THREADS")) nthreads = unsigned(std::atoi(e));
  const unsigned n = block.x * block.y * block.z;
  const unsigned nblocks = grid.x * grid.y * grid.z;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > nblocks) nthreads = nblocks;
  std::atomic<unsigned> next{0};
  auto worker = [&]() {
    gridDim = Index{grid.x, grid.y, grid.z};
    blockDim = Index{block.x, block.y, block.z};
    g_blk.body = &body;
    for (;;) {
      const unsigned b = next.fetch_add(1);
      if (b >= nblocks) break;
      blockIdx = Index{b % grid.x, (b / grid.x) % grid.y, b / (grid.x * grid.y)};
      run_block(n, block);
    }
  };
  std::vector<std::thread> pool;
  for (unsigned t = 0; t < nthreads; ++t) pool.emplace_back(worker);
  for (auto &t : pool) t.join();
}

// ---- wavefront operations ----

void op_readlane(const unsigned char (*ins)[64], unsigned char (*outs)[64], int src) {
  for (int l = 0; l < 64; ++l) std::memcpy(outs[l], ins[src], 64);
}

void op_shfl_xor(const unsigned char (*ins)[64], unsigned char (*outs)[64], int mask) {
  for (int l = 0; l < 64; ++l) std::memcpy(outs[l], ins[(l ^ mask) & 63], 64);
}

void check_dpp(int ctrl, int row_mask, int bank_mask) {
  if (ctrl < 0 || ctrl > 0xFF || row_mask != 0xF || bank_mask != 0xF)
    fail("DPP control other than quad_perm with all rows and banks");
}

void op_quad_perm(const unsigned char (*ins)[64], unsigned char (*outs)[64], int ctrl) {
  for (int l = 0; l < 64; ++l) std::memcpy(outs[l], ins[(l & ~3) + ((ctrl >> (2 * (l & 3))) & 3)], 64);
}

// 16 x 16 x K products: lane l supplies A[l % 16][k] and B[k][l % 16] for the
// k of its group l / 16 (one k for K = 4, eight consecutive for K = 32;
// any consistent assignment of k gives the same product). Output element v
// of lane l: column l % 16, row l / 16 + 4 v (FP64) or 4 (l / 16) + v (FP32).
void op_mfma_f64_16x16x4(const unsigned char (*ins)[64], unsigned char (*outs)[64], int) {
  const InF64 *in[64];
  for (int l = 0; l < 64; ++l) in[l] = reinterpret_cast<const InF64 *>(ins[l]);
  for (int l = 0; l < 64; ++l) {
    d4 r;
    for (int v = 0; v < 4; ++v) {
      const int i = l / 16 + 4 * v, j = l % 16;
      double acc = in[l]->c[v];
      for (int k = 0; k < 4; ++k) acc = std::fma(in[i + 16 * k]->a, in[j + 16 * k]->b, acc);
      r[v] = acc;
    }
    std::memcpy(outs[l], &r, sizeof(r));
  }
}

void op_mfma_f32_16x16x4(const unsigned char (*ins)[64], unsigned char (*outs)[64], int) {
  const InF32 *in[64];
  for (int l = 0; l < 64; ++l) in[l] = reinterpret_cast<const InF32 *>(ins[l]);
  for (int l = 0; l < 64; ++l) {
    f4 r;
    for (int v = 0; v < 4; ++v) {
      const int i = 4 * (l / 16) + v, j = l % 16;
      double acc = 0.0;
      for (int k = 0; k < 4; ++k) acc += double(in[i + 16 * k]->a) * double(in[j + 16 * k]->b);
      r[v] = float(acc + double(in[l]->c[v]));
    }
    std::memcpy(outs[l], &r, sizeof(r));
  }
}

void op_mfma_f32_16x16x32_bf16(const unsigned char (*ins)[64], unsigned char (*outs)[64], int) {
  const InBF16 *in[64];
  for (int l = 0; l < 64; ++l) in[l] = reinterpret_cast<const InBF16 *>(ins[l]);
  for (int l = 0; l < 64; ++l) {
    f4 r;
    for (int v = 0; v < 4; ++v) {
      const int i = 4 * (l / 16) + v, j = l % 16;
      double acc = 0.0;
      for (int g = 0; g < 4; ++g)
        for (int e = 0; e < 8; ++e)
          acc += double(float(in[i + 16 * g]->a[e])) * double(float(in[j + 16 * g]->b[e]));
      r[v] = float(acc + double(in[l]->c[v]));
    }
    std::memcpy(outs[l], &r, sizeof(r));
  }
}

}  // namespace emu

hipError_t hipGetLastError() { return hipSuccess; }

extern "C" unsigned long long emu_divergent_barriers() { return emu::g_divergent.load(); }
