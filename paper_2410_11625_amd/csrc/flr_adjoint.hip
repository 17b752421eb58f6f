// Window sums and a fixed-order reduction of FP64 planes, for the FLR adjoint.
//
// The adjoint recomputes the window moments as FP64 sums of anchored input
// products, and sums its per-pixel fields over the same clipped window (the
// window sum is its own adjoint). The window-sum tile is box_tile
// (flr_box.hpp): one workgroup per strip of kThreads input columns of one
// plane and segment of rows, running vertical sums per lane, horizontal sums
// by segmented prefixes.
#include <hip/hip_runtime.h>

#include "flr_box.hpp"
#include "flr_launch.hpp"
#include "flr_prefix.hpp"

namespace flr {

template <int SRC, bool WIDE, bool RING>
__global__ void __launch_bounds__(256) adj_box_kernel(AdjBoxArgs a) {
  box_tile<SRC, WIDE, RING>(a, blockIdx.x, blockIdx.y);
}

struct AdjPairArgs {
  const double* src;
  double* dst;
  int n;
};

__global__ void __launch_bounds__(256) adj_pair_sum_kernel(AdjPairArgs a) {
  extern __shared__ float lds[];
  double* part = reinterpret_cast<double*>(lds);  // [2][kThreads]
  const int tid = threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  for (int i = tid; i < a.n; i += kThreads) {
    s0 += a.src[2 * i];
    s1 += a.src[2 * i + 1];
  }
  part[tid] = s0;
  part[kThreads + tid] = s1;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (tid < s) {
      part[tid] += part[tid + s];
      part[kThreads + tid] += part[kThreads + tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    a.dst[0] = part[0];
    a.dst[1] = part[kThreads];
  }
}

template <bool WIDE, bool RING>
static void box_dispatch(const AdjBoxArgs& a, dim3 grid, size_t lds, hipStream_t s) {
  if (a.srcf)
    hipLaunchKernelGGL((adj_box_kernel<BOX_MEAN32, WIDE, RING>), grid, dim3(kThreads), lds, s, a);
  else if (a.src && a.count_first)  // count_first marks a mean of FP64 planes here
    hipLaunchKernelGGL((adj_box_kernel<BOX_MEAN64, WIDE, RING>), grid, dim3(kThreads), lds, s, a);
  else if (a.src)
    hipLaunchKernelGGL((adj_box_kernel<BOX_SUM64, WIDE, RING>), grid, dim3(kThreads), lds, s, a);
  else if (a.gout)
    hipLaunchKernelGGL((adj_box_kernel<BOX_AVGFIELDS, WIDE, RING>), grid, dim3(kThreads), lds, s,
                       a);
  else
    hipLaunchKernelGGL((adj_box_kernel<BOX_PRODUCTS, WIDE, RING>), grid, dim3(kThreads), lds, s,
                       a);
}

static hipError_t box_launch(AdjBoxArgs a, int planes, hipStream_t s) {
  // windows of up to 2r + 1 = 65 columns: at most two 64-lane prefix segments
  if (planes <= 0 || planes > 65535 || a.H < 1 || a.W < 1 || a.r < 0 || a.r > 32)
    return hipErrorInvalidValue;
  const dim3 grid(box_plan(a, planes), planes);
  a.ring = box_lds_bytes(a.r, true) <= kBoxLdsMax ? 1 : 0;
  const size_t lds = box_lds_bytes(a.r, a.ring != 0);
  if (wide_segments(a.r)) {
    if (a.ring)
      box_dispatch<true, true>(a, grid, lds, s);
    else
      box_dispatch<true, false>(a, grid, lds, s);
  } else {
    if (a.ring)
      box_dispatch<false, true>(a, grid, lds, s);
    else
      box_dispatch<false, false>(a, grid, lds, s);
  }
  return hipGetLastError();
}

hipError_t launch_mean_planes(const float* src, float* dst, int planes, int H, int W, int r,
                              hipStream_t s) {
  if (!src || !dst) return hipErrorInvalidValue;
  AdjBoxArgs a = {};
  a.srcf = src;
  a.dstf = dst;
  a.H = H;
  a.W = W;
  a.r = r;
  return box_launch(a, planes, s);
}

hipError_t launch_box(const double* src, double* dst, int planes, int H, int W, int r,
                      hipStream_t s) {
  if (!src) return hipErrorInvalidValue;
  AdjBoxArgs a = {};
  a.src = src;
  a.dst = dst;
  a.H = H;
  a.W = W;
  a.r = r;
  return box_launch(a, planes, s);
}

hipError_t launch_box_products(const float* guides, const float* noisy, int Q, int C, int H,
                               int W, int r, double* dst, hipStream_t s, bool with_count) {
  AdjBoxArgs a = {};
  a.guides = guides;
  a.noisy = noisy;
  a.dst = dst;
  a.H = H;
  a.W = W;
  a.r = r;
  a.Q = Q;
  a.C = C;
  a.count_first = with_count ? 1 : 0;
  return box_launch(a, num_sums(Q, C) + a.count_first, s);
}

hipError_t launch_box_avgfields(const float* guides, const float* gout, int Q, int C, int H,
                                int W, int r, double* dst, hipStream_t s) {
  if (!guides || !gout || !dst) return hipErrorInvalidValue;
  AdjBoxArgs a = {};
  a.guides = guides;
  a.gout = gout;
  a.dst = dst;
  a.H = H;
  a.W = W;
  a.r = r;
  a.Q = Q;
  a.C = C;
  return box_launch(a, C + Q * C, s);
}

hipError_t launch_mean_planes64(const double* src, double* dst, int planes, int H, int W, int r,
                                hipStream_t s) {
  if (!src || !dst) return hipErrorInvalidValue;
  AdjBoxArgs a = {};
  a.src = src;
  a.dst = dst;
  a.count_first = 1;
  a.H = H;
  a.W = W;
  a.r = r;
  return box_launch(a, planes, s);
}

hipError_t launch_pair_sum(const double* src, int n, double* dst, hipStream_t s) {
  if (n < 0) return hipErrorInvalidValue;
  AdjPairArgs a;
  a.src = src;
  a.dst = dst;
  a.n = n;
  hipLaunchKernelGGL(adj_pair_sum_kernel, dim3(1), dim3(kThreads), 2 * kThreads * sizeof(double), s,
                     a);
  return hipGetLastError();
}

}  // namespace flr
