// Separable Gaussian blur of the low-resolution moment planes of the
// downsampled-moment variant. A workgroup blurs one 16 x 16 tile of one
// plane: it stages the tile with an R-wide border in LDS (zero outside the
// grid), runs the pass along the rows into a second LDS buffer, then the
// pass along the columns.
#include <hip/hip_runtime.h>

#include "flr_launch.hpp"

namespace flr {

constexpr int kLrTile = 16;

struct LrBlurArgs {
  const double* src;
  double* dst;
  int Hl, Wl, R, tiles_x;
  double taps[2 * kMaxLowresRadius + 1];
};

__global__ void __launch_bounds__(256) lr_blur_kernel(LrBlurArgs a) {
  constexpr int SMAX = kLrTile + 2 * kMaxLowresRadius;
  __shared__ double tile[SMAX * SMAX];
  __shared__ double mid[SMAX * kLrTile];
  const int tid = threadIdx.x;
  const int R = a.R, S = kLrTile + 2 * R;
  const int bx = blockIdx.x % a.tiles_x, by = blockIdx.x / a.tiles_x;
  const int64_t pll = (int64_t)a.Hl * a.Wl;
  const double* src = a.src + (int64_t)blockIdx.y * pll;
  const int I0 = by * kLrTile - R, J0 = bx * kLrTile - R;
  // at most four items per lane (S <= 32); loads from clamped positions,
  // issued together, zero outside the grid
  double v[4];
  bool in[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int t = tid + u * kThreads;
    const int ii = t / S, jj = t - (t / S) * S;
    const int I = I0 + ii, J = J0 + jj;
    in[u] = t < S * S && I >= 0 && I < a.Hl && J >= 0 && J < a.Wl;
    const int Ic = I < 0 ? 0 : (I >= a.Hl ? a.Hl - 1 : I);
    const int Jc = J < 0 ? 0 : (J >= a.Wl ? a.Wl - 1 : J);
    v[u] = src[(int64_t)Ic * a.Wl + Jc];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int t = tid + u * kThreads;
    if (t < S * S) tile[t] = in[u] ? v[u] : 0.0;
  }
  __syncthreads();
  for (int t = tid; t < S * kLrTile; t += kThreads) {
    const int ii = t / kLrTile, jj = t - (t / kLrTile) * kLrTile;
    double s = 0.0;
    for (int d = -R; d <= R; ++d) s = fma(a.taps[d + R], tile[ii * S + jj + R + d], s);
    mid[t] = s;
  }
  __syncthreads();
  const int ii = tid / kLrTile, jj = tid - (tid / kLrTile) * kLrTile;
  const int I = by * kLrTile + ii, J = bx * kLrTile + jj;
  if (I < a.Hl && J < a.Wl) {
    double s = 0.0;
    for (int d = -R; d <= R; ++d) s = fma(a.taps[d + R], mid[(ii + R + d) * kLrTile + jj], s);
    a.dst[(int64_t)blockIdx.y * pll + (int64_t)I * a.Wl + J] = s;
  }
}

hipError_t launch_lr_blur(const double* src, double* dst, int planes, int Hl, int Wl, int R,
                          const double* taps, hipStream_t s) {
  if (planes <= 0 || planes > 65535 || Hl < 1 || Wl < 1 || R < 0 || R > kMaxLowresRadius)
    return hipErrorInvalidValue;
  LrBlurArgs a;
  a.src = src;
  a.dst = dst;
  a.Hl = Hl;
  a.Wl = Wl;
  a.R = R;
  a.tiles_x = (Wl + kLrTile - 1) / kLrTile;
  const int tiles_y = (Hl + kLrTile - 1) / kLrTile;
  for (int k = 0; k < 2 * kMaxLowresRadius + 1; ++k) a.taps[k] = k <= 2 * R ? taps[k] : 0.0;
  hipLaunchKernelGGL(lr_blur_kernel, dim3(a.tiles_x * tiles_y, planes), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace flr
