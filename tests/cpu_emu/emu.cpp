// Host execution of the FLR kernel sources, for CPU-side tests of their
// indexing, synchronisation and arithmetic. Compiled with g++ together with
// the library's own host dispatcher (flr_api.cpp), against the CPU stand-in
// for the HIP runtime in ./hip/hip_runtime.h. Test infrastructure only.
//
// * A workgroup runs on one host thread as blockDim.x user-space fibers
//   (ucontext), one per lane. __syncthreads() parks a lane until every lane
//   of the workgroup is parked there; a DPP move parks it until every lane
//   of its 64-lane wavefront has published its source value. Parking at
//   different barriers, or finishing while others wait, is reported as a
//   launch failure instead of hanging.
// * Workgroups run in parallel on several host threads, each with its own
//   LDS (a thread_local array). Before each workgroup the requested bytes
//   are filled with NaN (so reads of never-written LDS poison the result)
//   and the rest with a canary that is checked afterwards.
// * Each lane stack sits above a PROT_NONE guard page.
// * emu_alloc() places each buffer against a PROT_NONE guard page, so an
//   out-of-bounds global access past the end faults immediately.
#include <sys/mman.h>
#include <ucontext.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "hip/hip_runtime.h"

// AddressSanitizer builds: tell ASan about every switch between the
// scheduler's stack and a lane's fiber stack.
#if defined(__SANITIZE_ADDRESS__)
#include <sanitizer/common_interface_defs.h>
static inline void fiber_start(void** save, const void* bottom, size_t size) {
  __sanitizer_start_switch_fiber(save, bottom, size);
}
static inline void fiber_finish(void* save, const void** bottom_old, size_t* size_old) {
  __sanitizer_finish_switch_fiber(save, bottom_old, size_old);
}
#else
static inline void fiber_start(void**, const void*, size_t) {}
static inline void fiber_finish(void*, const void**, size_t*) {}
#endif

thread_local dim3 threadIdx;
thread_local dim3 blockIdx;
dim3 blockDim;
dim3 gridDim;

static hipError_t g_last = hipSuccess;
static char g_msg[256] = "";
static std::mutex g_err_mu;

static void set_error(hipError_t e, const char* msg) {
  std::lock_guard<std::mutex> lk(g_err_mu);
  if (g_last == hipSuccess) {
    g_last = e;
    std::snprintf(g_msg, sizeof g_msg, "%s", msg);
  }
}

hipError_t hipGetLastError() {
  const hipError_t e = g_last;
  g_last = hipSuccess;
  return e;
}

namespace {

constexpr unsigned kWave = 64;
#if defined(__SANITIZE_ADDRESS__)
// ASan clears the shadow of a fiber's whole stack at every switch into it:
// smaller stacks keep that a short memset
constexpr size_t kStackBytes = 128 * 1024;
#else
constexpr size_t kStackBytes = 512 * 1024;
#endif

enum LaneState : int { READY, AT_BLOCK_BARRIER, AT_WAVE_BARRIER, DONE };

struct Lane {
  ucontext_t ctx;
  LaneState state;
  unsigned dpp_calls;
  unsigned mfma_calls;
  char* stack;  // kStackBytes above one guard page
  void* fake = nullptr;  // ASan fake-stack handle while switched out
};

// One host thread's workgroup scheduler.
struct Workgroup {
  ucontext_t sched;
  const void* sched_bottom = nullptr;  // the scheduler's (thread's) stack, for ASan
  size_t sched_size = 0;
  void* sched_fake = nullptr;
  std::vector<Lane> lanes;
  unsigned cur = 0;
  int dpp[2][1024];
  uint16_t mfa[2][1024][4], mfb[2][1024][4];
  std::function<void()> body;

  Workgroup() : lanes(1024) {
    const size_t pg = (size_t)sysconf(_SC_PAGESIZE);
    for (auto& l : lanes) {
      char* base = static_cast<char*>(mmap(nullptr, kStackBytes + pg, PROT_READ | PROT_WRITE,
                                           MAP_PRIVATE | MAP_ANONYMOUS, -1, 0));
      if (base == MAP_FAILED) std::abort();
      mprotect(base, pg, PROT_NONE);
      l.stack = base + pg;
    }
  }
  ~Workgroup() {
    const size_t pg = (size_t)sysconf(_SC_PAGESIZE);
    for (auto& l : lanes) munmap(l.stack - pg, kStackBytes + pg);
  }

  void park(LaneState s) {
    Lane& l = lanes[cur];
    l.state = s;
    fiber_start(&l.fake, sched_bottom, sched_size);
    swapcontext(&l.ctx, &sched);
    fiber_finish(l.fake, nullptr, nullptr);
  }

  static void entry();

  // Runs `n` lanes of block `b` to completion; false on a barrier mismatch.
  bool run(unsigned n, dim3 b, char* err, size_t errn) {
    for (unsigned t = 0; t < n; ++t) {
      Lane& l = lanes[t];
      getcontext(&l.ctx);
      l.ctx.uc_stack.ss_sp = l.stack;
      l.ctx.uc_stack.ss_size = kStackBytes;
      l.ctx.uc_link = &sched;
      makecontext(&l.ctx, entry, 0);
      l.state = READY;
      l.dpp_calls = 0;
      l.mfma_calls = 0;
    }
    blockIdx = b;
    for (;;) {
      for (unsigned t = 0; t < n; ++t) {
        if (lanes[t].state != READY) continue;
        cur = t;
        threadIdx = dim3(t);
        fiber_start(&sched_fake, lanes[t].stack, kStackBytes);
        swapcontext(&sched, &lanes[t].ctx);
        fiber_finish(sched_fake, nullptr, nullptr);
      }
      unsigned done = 0, at_block = 0;
      bool released = false;
      for (unsigned w0 = 0; w0 < n; w0 += kWave) {
        const unsigned w1 = std::min(n, w0 + kWave);
        unsigned at_wave = 0;
        for (unsigned t = w0; t < w1; ++t) at_wave += lanes[t].state == AT_WAVE_BARRIER;
        if (at_wave == w1 - w0) {
          for (unsigned t = w0; t < w1; ++t) lanes[t].state = READY;
          released = true;
        }
      }
      if (released) continue;
      for (unsigned t = 0; t < n; ++t) {
        done += lanes[t].state == DONE;
        at_block += lanes[t].state == AT_BLOCK_BARRIER;
      }
      if (done == n) return true;
      if (at_block == n) {
        for (unsigned t = 0; t < n; ++t) lanes[t].state = READY;
        continue;
      }
      std::snprintf(err, errn,
                    "block (%u,%u): lanes diverged at barriers (%u done, %u at the workgroup "
                    "barrier)", b.x, b.y, done, at_block);
      return false;
    }
  }
};

thread_local Workgroup* t_wg = nullptr;

void Workgroup::entry() {
  Workgroup* w = t_wg;
  fiber_finish(nullptr, &w->sched_bottom, &w->sched_size);
  w->body();
  w->lanes[w->cur].state = DONE;
  fiber_start(nullptr, w->sched_bottom, w->sched_size);  // this fiber ends here
}

}  // namespace

void __syncthreads() { t_wg->park(AT_BLOCK_BARRIER); }

int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask,
                                bool bound_ctrl) {
  Workgroup* wg = t_wg;
  const unsigned t = wg->cur, w = t / kWave, l = t % kWave;
  const unsigned slot = wg->lanes[t].dpp_calls++ & 1u;
  wg->dpp[slot][t] = src;
  wg->park(AT_WAVE_BARRIER);
  const int row = (int)(l / 16), rl = (int)(l % 16);
  if (!((row_mask >> row) & 1) || !((bank_mask >> (rl / 4)) & 1)) return old;
  int s = -1;
  if (ctrl >= 0 && ctrl <= 0xff) {  // quad_perm: lane 4q + i reads 4q + sel_i
    s = (int)(l & ~3u) + ((ctrl >> (2 * (rl & 3))) & 3);
  } else if (ctrl == 0x140) {  // row_mirror
    s = row * 16 + (15 - rl);
  } else if (ctrl == 0x141) {  // row_half_mirror
    s = row * 16 + (rl & 8) + (7 - (rl & 7));
  } else if (ctrl > 0x100 && ctrl <= 0x10f) {  // row_shl:k
    const int k = ctrl - 0x100;
    s = rl + k <= 15 ? (int)l + k : -1;
  } else if (ctrl > 0x120 && ctrl <= 0x12f) {  // row_ror:k
    const int k = ctrl - 0x120;
    s = row * 16 + ((rl - k + 16) & 15);
  } else if (ctrl > 0x110 && ctrl <= 0x11f) {
    const int k = ctrl - 0x110;
    s = rl >= k ? (int)l - k : -1;
  } else if (ctrl == 0x138) {  // wave_shr:1
    s = l >= 1 ? (int)l - 1 : -1;
  } else if (ctrl == 0x142) {
    s = row >= 1 ? (row - 1) * 16 + 15 : -1;
  } else if (ctrl == 0x143) {
    s = row >= 2 ? 31 : -1;
  } else {
    std::fprintf(stderr, "emulator: unsupported DPP control 0x%x\n", ctrl);
    std::abort();
  }
  if (s < 0) return bound_ctrl ? 0 : old;
  return wg->dpp[slot][w * kWave + (unsigned)s];
}

unsigned __builtin_amdgcn_raw_buffer_load_b32(__amdgpu_buffer_rsrc_t r, int vo, int so, int) {
  const long long o = (long long)vo + (long long)so;
  if (vo < 0 || so < 0 || o + 4 > (long long)r.bytes) {
    std::fprintf(stderr, "emulator: buffer load at %lld outside [0, %d)\n", o, r.bytes);
    std::abort();
  }
  unsigned v;
  std::memcpy(&v, r.base + o, sizeof v);
  return v;
}

emu_f32x4 __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(emu_bf16x4 a, emu_bf16x4 b, emu_f32x4 c, int,
                                                    int, int) {
  Workgroup* wg = t_wg;
  const unsigned t = wg->cur, w0 = t / kWave * kWave, l = t % kWave;
  const unsigned slot = wg->lanes[t].mfma_calls++ & 1u;
  for (int j = 0; j < 4; ++j) {
    wg->mfa[slot][t][j] = (uint16_t)a[j];
    wg->mfb[slot][t][j] = (uint16_t)b[j];
  }
  wg->park(AT_WAVE_BARRIER);
  auto bf = [](uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, sizeof f);
    return (double)f;
  };
  emu_f32x4 d;
  const unsigned n = l % 16;
  for (int i = 0; i < 4; ++i) {
    const unsigned m = 4 * (l / 16) + i;
    double acc = c[i];
    for (unsigned k = 0; k < 16; ++k)
      acc += bf(wg->mfa[slot][w0 + m + 16 * (k / 4)][k % 4]) * bf(wg->mfb[slot][w0 + n + 16 * (k / 4)][k % 4]);
    d[i] = (float)acc;
  }
  return d;
}

namespace flr {
constexpr size_t kEmuLdsFloats = 163840 / 4 + 4096;
alignas(64) thread_local float lds[kEmuLdsFloats];
}  // namespace flr

static const uint32_t kCanary = 0x7fc0dead;

void emu_launch_erased(void (*tramp)(const void*, const void*), const void* kernel,
                       const void* arg, dim3 grid, dim3 block, size_t lds_bytes) {
  if (lds_bytes > 163840 || block.x == 0 || block.x > 1024) {
    set_error(hipErrorInvalidValue, "bad launch shape");
    return;
  }
  blockDim = block;
  gridDim = grid;
  const size_t used = (lds_bytes + 3) / 4;
  std::atomic<unsigned> next{0};
  std::atomic<bool> failed{false};
  auto worker = [&]() {
    Workgroup wg;
    t_wg = &wg;
    wg.body = [&]() { tramp(kernel, arg); };
    char err[200];
    for (unsigned b; !failed && (b = next++) < grid.x * grid.y;) {
      uint32_t* w = reinterpret_cast<uint32_t*>(flr::lds);
      for (size_t i = 0; i < used; ++i) w[i] = 0x7fc00000u;  // quiet NaN
      for (size_t i = used; i < flr::kEmuLdsFloats; ++i) w[i] = kCanary;
      if (!wg.run(block.x, dim3(b % grid.x, b / grid.x), err, sizeof err)) {
        set_error(hipErrorLaunchFailure, err);
        failed = true;
        break;
      }
      for (size_t i = used; i < flr::kEmuLdsFloats; ++i) {
        if (w[i] != kCanary) {
          std::snprintf(err, sizeof err, "LDS write past %zu bytes at float %zu (block %u)",
                        lds_bytes, i, b);
          set_error(hipErrorLaunchFailure, err);
          failed = true;
          break;
        }
      }
    }
    t_wg = nullptr;
  };
  const unsigned hw = std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
  const unsigned nt = std::min(hw, grid.x * grid.y);
  std::vector<std::thread> ts;
  for (unsigned i = 0; i < nt; ++i) ts.emplace_back(worker);
  for (auto& th : ts) th.join();
}

#include "flr_device.hpp"

// The emulator instantiates a subset of guide counts; others report an error.
FLR_DEFINE_Q(1)
FLR_DEFINE_Q(2)
FLR_DEFINE_Q(3)
FLR_DEFINE_Q(4)
FLR_DEFINE_Q(8)
#define FLR_EMU_STUB(q)                                                        \
  namespace flr {                                                              \
  hipError_t launch_q##q(int, int, const LaunchArgs&, hipStream_t) {           \
    std::snprintf(g_msg, sizeof g_msg, "Q=%d not instantiated in emulator", q); \
    return hipErrorInvalidValue;                                               \
  }                                                                            \
  }
FLR_EMU_STUB(5)
FLR_EMU_STUB(6)
FLR_EMU_STUB(7)
FLR_EMU_STUB(9)
FLR_EMU_STUB(10)
FLR_EMU_STUB(11)
FLR_EMU_STUB(12)

extern "C" {

const char* emu_message() { return g_msg; }

// Buffer of `bytes` (rounded up to 16) whose end touches a PROT_NONE page and
// which is preceded by one.
void* emu_alloc(size_t bytes) {
  const size_t pg = (size_t)sysconf(_SC_PAGESIZE);
  const size_t nb = (bytes + 15) & ~(size_t)15;
  const size_t data = (nb + pg - 1) / pg * pg;
  char* base = static_cast<char*>(
      mmap(nullptr, data + 2 * pg, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0));
  if (base == MAP_FAILED) return nullptr;
  mprotect(base, pg, PROT_NONE);
  mprotect(base + pg + data, pg, PROT_NONE);
  return base + pg + data - nb;
}

void emu_free(void* p, size_t bytes) {
  if (!p) return;
  const size_t pg = (size_t)sysconf(_SC_PAGESIZE);
  const size_t nb = (bytes + 15) & ~(size_t)15;
  const size_t data = (nb + pg - 1) / pg * pg;
  char* base = static_cast<char*>(p) - (data - nb) - pg;
  munmap(base, data + 2 * pg);
}

}  // extern "C"
