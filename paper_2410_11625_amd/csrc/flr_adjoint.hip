// Window sums and a fixed-order reduction of FP64 planes, for the FLR adjoint.
//
// The adjoint recomputes the window moments as FP64 sums of anchored input
// products, and sums its per-pixel fields over the same clipped window (the
// window sum is its own adjoint). One workgroup owns
// a strip of kThreads input columns (kThreads - 2r output columns) of one
// plane and walks down a segment of rows: each lane keeps the running
// vertical sum of its column (add the row entering the window, subtract the
// row leaving it), stages it in LDS, and the lanes that own output columns
// add the 2r+1 staged values of their window. Columns outside the image
// stage 0, which clips the window at the left and right borders.
#include <hip/hip_runtime.h>

#include "flr_launch.hpp"

namespace flr {

constexpr int kBoxSegRows = 64;

struct AdjBoxArgs {
  const float* srcf;   // BOX_MEAN32: FP32 planes, averaged into dstf
  float* dstf;
  const double* src;   // FP64 planes, or NULL for the product channels below
  const float* guides; // product channels: guides [Q][H][W]
  const float* noisy;  // product channels: noisy [C][H][W]
  double* dst;
  int64_t plane;  // elements per plane
  int H, W, r, seg_rows, tiles_x;
  int Q, C;
  int count_first;  // BOX_PRODUCTS: plane 0 is the window pixel count, channels follow
};

// Input plane v of the product channels: a guide (v < Q) or a noisy channel.
__device__ __forceinline__ const float* input_plane(const AdjBoxArgs& a, int v) {
  return v < a.Q ? a.guides + (int64_t)v * a.plane : a.noisy + (int64_t)(v - a.Q) * a.plane;
}

// Factors of product channel ch in the moment order g_q | y_c | g_p g_q
// (p <= q) | g_q y_c: input planes u and v (v = -1 for a first moment).
__device__ __forceinline__ void channel_factors(int ch, int Q, int C, int* u, int* v) {
  if (ch < Q + C) {
    *u = ch;
    *v = -1;
    return;
  }
  ch -= Q + C;
  const int np = Q * (Q + 1) / 2;
  if (ch < np) {
    int p = 0;
    while (ch >= Q - p) {
      ch -= Q - p;
      ++p;
    }
    *u = p;
    *v = p + ch;
    return;
  }
  ch -= np;
  *u = ch / C;
  *v = Q + ch % C;
}

// Window sums of FP64 planes (BOX_SUM64), of the anchored products of the
// inputs (BOX_PRODUCTS: channel blockIdx.y is (x_u - c_u)(x_v - c_v) or
// x_u - c_u, with c the plane's value at pixel (0, 0)), or window means of
// FP32 planes (BOX_MEAN32: FP64 sums divided by the pixel count).
enum BoxSource : int { BOX_SUM64 = 0, BOX_PRODUCTS = 1, BOX_MEAN32 = 2, BOX_MEAN64 = 3 };

template <int SRC>
__global__ void __launch_bounds__(256) adj_box_kernel(AdjBoxArgs a) {
  constexpr bool PRODUCTS = SRC == BOX_PRODUCTS;
  extern __shared__ float lds[];
  double* rows = reinterpret_cast<double*>(lds);  // two rows of kThreads
  const int tid = threadIdx.x;
  const int r = a.r, H = a.H, W = a.W;
  const int tile = blockIdx.x % a.tiles_x, seg = blockIdx.x / a.tiles_x;
  const int x = tile * (kThreads - 2 * r) - r + tid;
  const bool inx = x >= 0 && x < W;
  const int y0 = seg * a.seg_rows;
  const int y1 = y0 + a.seg_rows < H ? y0 + a.seg_rows : H;
  const int64_t col = inx ? x : 0;
  const double* src = nullptr;
  const float* srcf = nullptr;
  const float *pu = nullptr, *pv = nullptr;
  double cu = 0.0, cv = 0.0;
  bool single = false;  // a first moment: the second factor is 1
  bool ones = false;    // the pixel count: every factor is 1
  if constexpr (PRODUCTS) {
    int u, v;
    const int ch = (int)blockIdx.y - a.count_first;
    ones = ch < 0;
    channel_factors(ones ? 0 : ch, a.Q, a.C, &u, &v);
    single = v < 0;
    pu = input_plane(a, u);
    pv = single ? pu : input_plane(a, v);  // read either way, used only for products
    cu = pu[0];
    cv = pv[0];
    pu += col;
    pv += col;
  } else if constexpr (SRC == BOX_MEAN32) {
    srcf = a.srcf + (int64_t)blockIdx.y * a.plane + col;
  } else {  // BOX_SUM64, BOX_MEAN64
    src = a.src + (int64_t)blockIdx.y * a.plane + col;
  }
  auto value = [&](int yy) -> double {
    if constexpr (PRODUCTS) {
      const double t = (double)pu[(int64_t)yy * W] - cu;
      const double w = (double)pv[(int64_t)yy * W] - cv;
      return ones ? 1.0 : (single ? t : t * w);
    } else if constexpr (SRC == BOX_MEAN32) {
      return (double)srcf[(int64_t)yy * W];
    } else {  // BOX_SUM64, BOX_MEAN64
      return src[(int64_t)yy * W];
    }
  };
  auto clamp_row = [&](int yy) { return yy < 0 ? 0 : (yy >= H ? H - 1 : yy); };
  double* dst = SRC == BOX_MEAN32 ? nullptr : a.dst + (int64_t)blockIdx.y * a.plane;  // FP64 out
  const bool owner = inx && tid >= r && tid < kThreads - r;
  // Loads are unconditional from clamped rows and masked afterwards, in
  // batches of kRowBatch rows, so that a batch's loads are in flight
  // together instead of one round trip per row.
  constexpr int kRowBatch = 8;
  double v = 0.0;
  {
    const int lo = y0 - r, hi = y0 + r;
    for (int yb = lo; yb <= hi; yb += kRowBatch) {
      double t[kRowBatch];
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) t[u] = value(clamp_row(yb + u));
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
        const int yy = yb + u;
        v += (inx && yy <= hi && yy >= 0 && yy < H) ? t[u] : 0.0;
      }
    }
  }
  for (int yc = y0; yc < y1; yc += kRowBatch) {
    double ent[kRowBatch], lea[kRowBatch];
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {
      const int y = yc + u;
      const bool step = inx && y > y0 && y < y1;
      const double e = value(clamp_row(y + r));
      const double l = value(clamp_row(y - r - 1));
      ent[u] = step && y + r < H ? e : 0.0;
      lea[u] = step && y - r - 1 >= 0 ? l : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {
      const int y = yc + u;
      if (y >= y1) break;  // uniform across the workgroup
      v += ent[u] - lea[u];
      // alternate buffers: one barrier per row orders this row's writes
      // before its reads, and the reads of two rows back before these writes
      double* buf = rows + ((y - y0) & 1) * kThreads;
      buf[tid] = v;
      __syncthreads();
      if (owner) {
        double s = 0.0;
        for (int d = -r; d <= r; ++d) s += buf[tid + d];
        if constexpr (SRC == BOX_MEAN32 || SRC == BOX_MEAN64) {
          const int ny = (y + r < H - 1 ? y + r : H - 1) - (y - r > 0 ? y - r : 0) + 1;
          const int nx = (x + r < W - 1 ? x + r : W - 1) - (x - r > 0 ? x - r : 0) + 1;
          const double m = s / (double)(ny * nx);
          if constexpr (SRC == BOX_MEAN32)
            a.dstf[(int64_t)blockIdx.y * a.plane + (int64_t)y * W + x] = (float)m;
          else
            dst[(int64_t)y * W + x] = m;
        } else {
          dst[(int64_t)y * W + x] = s;
        }
      }
    }
  }
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

static hipError_t box_launch(AdjBoxArgs a, int planes, hipStream_t s) {
  if (planes <= 0 || planes > 65535 || a.H < 1 || a.W < 1 || a.r < 0 || 2 * a.r >= kThreads)
    return hipErrorInvalidValue;
  a.plane = (int64_t)a.H * a.W;
  a.seg_rows = kBoxSegRows < a.H ? kBoxSegRows : a.H;
  a.tiles_x = (a.W + (kThreads - 2 * a.r) - 1) / (kThreads - 2 * a.r);
  const int n_seg = (a.H + a.seg_rows - 1) / a.seg_rows;
  const dim3 grid(a.tiles_x * n_seg, planes);
  const size_t lds = 2 * kThreads * sizeof(double);
  if (a.srcf)
    hipLaunchKernelGGL(adj_box_kernel<BOX_MEAN32>, grid, dim3(kThreads), lds, s, a);
  else if (a.src && a.count_first)  // count_first marks a mean of FP64 planes here
    hipLaunchKernelGGL(adj_box_kernel<BOX_MEAN64>, grid, dim3(kThreads), lds, s, a);
  else if (a.src)
    hipLaunchKernelGGL(adj_box_kernel<BOX_SUM64>, grid, dim3(kThreads), lds, s, a);
  else
    hipLaunchKernelGGL(adj_box_kernel<BOX_PRODUCTS>, grid, dim3(kThreads), lds, s, a);
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
