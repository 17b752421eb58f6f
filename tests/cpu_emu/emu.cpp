// Host execution of the FLR kernel sources, for CPU-side tests of their
// indexing, synchronisation and arithmetic. Compiled with g++ together with
// the library's own host dispatcher (flr_api.cpp), against the CPU stand-in
// for the HIP runtime in ./hip/hip_runtime.h. Test infrastructure only.
//
// * A workgroup runs as blockDim.x std::threads meeting at a std::barrier.
// * LDS is one static array; before each workgroup the requested bytes are
//   filled with NaN (so reads of never-written LDS poison the result) and
//   the rest with a canary that is checked afterwards.
// * emu_alloc() places each buffer against a PROT_NONE guard page, so an
//   out-of-bounds global access past the end faults immediately.
#include <sys/mman.h>
#include <unistd.h>

#include <barrier>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "hip/hip_runtime.h"

thread_local dim3 threadIdx;
thread_local dim3 blockIdx;
dim3 blockDim;
dim3 gridDim;

static std::barrier<>* g_bar = nullptr;
static hipError_t g_last = hipSuccess;
static char g_msg[256] = "";

void __syncthreads() { g_bar->arrive_and_wait(); }

hipError_t hipGetLastError() {
  const hipError_t e = g_last;
  g_last = hipSuccess;
  return e;
}

namespace flr {
constexpr size_t kEmuLdsFloats = 163840 / 4 + 4096;
alignas(64) float lds[kEmuLdsFloats];
}  // namespace flr

static const uint32_t kCanary = 0x7fc0dead;

template <typename A>
void emu_launch_kernel(void (*k)(A), dim3 grid, dim3 block, size_t lds_bytes, hipStream_t, A a) {
  if (lds_bytes > 163840 || block.x == 0 || block.x > 1024) {
    g_last = hipErrorInvalidValue;
    return;
  }
  blockDim = block;
  gridDim = grid;
  const size_t used = (lds_bytes + 3) / 4;
  for (unsigned b = 0; b < grid.x; ++b) {
    uint32_t* w = reinterpret_cast<uint32_t*>(flr::lds);
    for (size_t i = 0; i < used; ++i) w[i] = 0x7fc00000u;  // quiet NaN
    for (size_t i = used; i < flr::kEmuLdsFloats; ++i) w[i] = kCanary;
    std::barrier<> bar((std::ptrdiff_t)block.x);
    g_bar = &bar;
    std::vector<std::thread> ts;
    ts.reserve(block.x);
    for (unsigned t = 0; t < block.x; ++t) {
      ts.emplace_back([=]() {
        threadIdx = dim3(t);
        blockIdx = dim3(b);
        k(a);
      });
    }
    for (auto& th : ts) th.join();
    for (size_t i = used; i < flr::kEmuLdsFloats; ++i) {
      if (w[i] != kCanary) {
        std::snprintf(g_msg, sizeof g_msg, "LDS write past %zu bytes at float %zu (block %u)",
                      lds_bytes, i, b);
        g_last = hipErrorLaunchFailure;
        return;
      }
    }
  }
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
