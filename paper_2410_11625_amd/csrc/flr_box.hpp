// Window sums of FP64 planes, of anchored input products, or window means
// (one workgroup's tile): the box passes of the FLR adjoint and of the
// joint frames of a batch.
#pragma once

#include <hip/hip_runtime.h>

#include "flr_launch.hpp"

namespace flr {



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
// inputs (BOX_PRODUCTS: channel `by` is (x_u - c_u)(x_v - c_v) or
// x_u - c_u, with c the plane's value at pixel (0, 0)), or window means of
// FP32 planes (BOX_MEAN32: FP64 sums divided by the pixel count).
enum BoxSource : int { BOX_SUM64 = 0, BOX_PRODUCTS = 1, BOX_MEAN32 = 2, BOX_MEAN64 = 3 };

template <int SRC>
__device__ __forceinline__ void box_tile(const AdjBoxArgs a, const int bx, const int by) {
  constexpr bool PRODUCTS = SRC == BOX_PRODUCTS;
  extern __shared__ float lds[];
  double* rows = reinterpret_cast<double*>(lds);  // two rows of kThreads
  const int tid = threadIdx.x;
  const int r = a.r, H = a.H, W = a.W;
  const int tile = bx % a.tiles_x, seg = bx / a.tiles_x;
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
    const int ch = by - a.count_first;
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
    srcf = a.srcf + (int64_t)by * a.plane + col;
  } else {  // BOX_SUM64, BOX_MEAN64
    src = a.src + (int64_t)by * a.plane + col;
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
  double* dst = SRC == BOX_MEAN32 ? nullptr : a.dst + (int64_t)by * a.plane;  // FP64 out
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
            a.dstf[(int64_t)by * a.plane + (int64_t)y * W + x] = (float)m;
          else
            dst[(int64_t)y * W + x] = m;
        } else {
          dst[(int64_t)y * W + x] = s;
        }
      }
    }
  }
}

}  // namespace flr
