// CPU stand-in for the few HIP runtime names the FLR kernel sources use, so
// that the same sources can be compiled with g++ and executed on the host:
// a workgroup runs as blockDim.x fibers on one host thread.
// Test infrastructure only.
#pragma once

#include <algorithm>
#include <chrono>
#include <thread>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ thread_local
#define HIP_SYMBOL(x) (&(x))

struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

struct alignas(8) uint2 {
  unsigned x, y;
};
struct alignas(16) uint4 {
  unsigned x, y, z, w;
};
struct alignas(16) float4 {
  float x, y, z, w;
};

extern thread_local dim3 threadIdx;
extern thread_local dim3 blockIdx;
extern dim3 blockDim;
extern dim3 gridDim;
void __syncthreads();

inline float rsqrtf(float x) { return 1.0f / std::sqrt(x); }

inline long long __double_as_longlong(double x) {
  long long v;
  std::memcpy(&v, &x, sizeof v);
  return v;
}
inline double __longlong_as_double(long long v) {
  double x;
  std::memcpy(&x, &v, sizeof x);
  return x;
}
inline int __float_as_int(float x) {
  int v;
  std::memcpy(&v, &x, sizeof v);
  return v;
}
inline float __int_as_float(int v) {
  float x;
  std::memcpy(&x, &v, sizeof x);
  return x;
}

inline unsigned __float_as_uint(float x) {
  unsigned v;
  std::memcpy(&v, &x, sizeof v);
  return v;
}
inline float __uint_as_float(unsigned v) {
  float x;
  std::memcpy(&x, &v, sizeof x);
  return x;
}

// Raw buffer descriptor and dword load. Kernels must keep every access
// inside the descriptor's range; the emulator aborts otherwise.
struct __amdgpu_buffer_rsrc_t {
  const char* base;
  int bytes;
};
inline __amdgpu_buffer_rsrc_t __builtin_amdgcn_make_buffer_rsrc(void* p, short stride, int bytes,
                                                               int) {
  if (stride != 0) std::abort();
  return {static_cast<const char*>(p), bytes};
}
unsigned __builtin_amdgcn_raw_buffer_load_b32(__amdgpu_buffer_rsrc_t r, int vo, int so, int aux);

inline void __builtin_amdgcn_sched_barrier(int) {}
inline int __builtin_amdgcn_readfirstlane(int v) { return v; }

// v_mfma_f32_16x16x16_bf16 of a 64-lane wavefront: D = C + A B with A 16x16
// (lane l: row l%16, k = 4*(l/16)..+3), B 16x16 (lane l: k = 4*(l/16)..+3,
// column l%16), C/D (lane l: rows 4*(l/16)..+3, column l%16). Every lane of
// the wavefront must call it at the same point.
typedef short emu_bf16x4 __attribute__((vector_size(8)));
typedef float emu_f32x4 __attribute__((vector_size(16)));
emu_f32x4 __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(emu_bf16x4 a, emu_bf16x4 b, emu_f32x4 c, int,
                                                    int, int);

// DPP lane move of a 64-lane wavefront (quad_perm, row_mirror,
// row_half_mirror, row_shl:1..15, row_shr:1..15, row_ror:1..15, wave_shr:1,
// row_bcast:15, row_bcast:31);
// every lane of the wavefront must call it at the same point.
int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask,
                                bool bound_ctrl);
using std::max;
using std::min;

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorLaunchFailure = 2 };
typedef void* hipStream_t;
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 0 };
inline hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }
hipError_t hipGetLastError();
enum hipMemcpyKind { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2 };
inline hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind) {
  std::memcpy(dst, src, n);
  return hipSuccess;
}
inline hipError_t hipMemset(void* dst, int v, size_t n) {
  std::memset(dst, v, n);
  return hipSuccess;
}
// Device atomics and fences of the persistent kernels: workgroups run on
// several host threads, so these are real atomics. (clang has the
// __hip_atomic_* builtins for the host too; the sanitizer build uses it.)
#ifndef __HIP_MEMORY_SCOPE_AGENT
#define __HIP_MEMORY_SCOPE_AGENT 3
#endif
inline int atomicAdd(int* p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline int atomicOr(int* p, int v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
#if !__has_builtin(__hip_atomic_load)
inline int __hip_atomic_load(const int* p, int, int) { return __atomic_load_n(p, __ATOMIC_SEQ_CST); }
#endif
#if !__has_builtin(__hip_atomic_fetch_add)
inline int __hip_atomic_fetch_add(int* p, int v, int, int) {
  return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}
#endif
inline void __builtin_amdgcn_fence(int, const char*) { __atomic_thread_fence(__ATOMIC_SEQ_CST); }
// a short real sleep: emulated workgroups are slow, and a spin-wait's
// iteration limit must outlast them
inline void __builtin_amdgcn_s_sleep(int) { std::this_thread::sleep_for(std::chrono::microseconds(20)); }

// Runs a kernel over the grid on host threads (defined by the emulator):
// `tramp(kernel, arg)` executes one lane.
void emu_launch_erased(void (*tramp)(const void*, const void*), const void* kernel,
                       const void* arg, dim3 grid, dim3 block, size_t lds_bytes);
template <typename A>
void emu_launch_kernel(void (*k)(A), dim3 grid, dim3 block, size_t lds_bytes, hipStream_t, A a) {
  emu_launch_erased(
      [](const void* kf, const void* ap) {
        reinterpret_cast<void (*)(A)>(const_cast<void*>(kf))(*static_cast<const A*>(ap));
      },
      reinterpret_cast<const void*>(k), &a, grid, block, lds_bytes);
}

#define hipLaunchKernelGGL(kernel, grid, block, lds, stream, ...) \
  emu_launch_kernel(kernel, dim3(grid), dim3(block), (size_t)(lds), (hipStream_t)(stream), __VA_ARGS__)
