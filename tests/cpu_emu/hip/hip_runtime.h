// CPU stand-in for the few HIP runtime names the FLR kernel sources use, so
// that the same sources can be compiled with g++ and executed on the host:
// a workgroup runs as blockDim.x host threads that meet at a real barrier.
// Test infrastructure only.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__
#define HIP_SYMBOL(x) (&(x))

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

extern thread_local dim3 threadIdx;
extern thread_local dim3 blockIdx;
extern dim3 blockDim;
extern dim3 gridDim;
void __syncthreads();

inline float rsqrtf(float x) { return 1.0f / std::sqrt(x); }
using std::max;
using std::min;

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorLaunchFailure = 2 };
typedef void* hipStream_t;
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 0 };
inline hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }
hipError_t hipGetLastError();

// Runs kernel `k` over the grid on host threads (defined by the emulator).
template <typename A>
void emu_launch_kernel(void (*k)(A), dim3 grid, dim3 block, size_t lds_bytes, hipStream_t, A a);

#define hipLaunchKernelGGL(kernel, grid, block, lds, stream, ...) \
  emu_launch_kernel(kernel, dim3(grid), dim3(block), (size_t)(lds), (hipStream_t)(stream), __VA_ARGS__)
