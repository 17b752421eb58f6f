// Window sums of FP64 planes, of anchored input products, or window means
// (one workgroup's tile): the box passes of the FLR adjoint and of the
// joint frames of a batch.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "flr_launch.hpp"
#include "flr_prefix.hpp"

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
// x_u - c_u, with c the plane's value at pixel (0, 0)), of the adjoint's
// averaging products (BOX_AVGFIELDS: plane `by` is G_c / n or
// (g_q - c_q) G_c / n, n the pixel's window count), or window means of
// FP32 or FP64 planes (BOX_MEAN32, BOX_MEAN64: FP64 sums divided by the
// pixel count).
//
// One workgroup: a strip of kThreads input columns (kThreads - 2r output
// columns) of one plane, walking down a segment of rows. Each lane keeps
// the running vertical sum of its column: it adds the row entering the
// window and subtracts the row leaving it, which (a.ring) it takes from a
// per-lane ring of the last 2r + 1 entering values in LDS instead of
// loading it again. The horizontal sum is the segmented prefix of the
// vertical sums (DPP moves) staged in LDS, three reads per output. Columns
// outside the image contribute 0, which clips the window at the left and
// right borders. WIDE: 64-lane prefix segments (r > 8).
enum BoxSource : int {
  BOX_SUM64 = 0,
  BOX_PRODUCTS = 1,
  BOX_MEAN32 = 2,
  BOX_MEAN64 = 3,
  BOX_AVGFIELDS = 4
};

template <int SRC, bool WIDE, bool RING>
__device__ __forceinline__ void box_tile(const AdjBoxArgs a, const int bx, const int by) {
  constexpr bool PRODUCTS = SRC == BOX_PRODUCTS || SRC == BOX_AVGFIELDS;
  constexpr bool F64 = SRC == BOX_SUM64 || SRC == BOX_MEAN64;
  using raw_t = typename std::conditional<F64, double, float>::type;
  extern __shared__ float lds[];
  // two prefix rows of kThreads + 1 (the last column is a zero pad), then
  // the ring: (2r + 1) rows of kThreads
  double* rows = reinterpret_cast<double*>(lds);
  double* ring = rows + 2 * (kThreads + 1) + threadIdx.x;
  const int tid = threadIdx.x;
  const int r = a.r, H = a.H, W = a.W;
  const int tile = bx % a.tiles_x, seg = bx / a.tiles_x;
  const int x = tile * (kThreads - 2 * r) - r + tid;
  const bool inx = x >= 0 && x < W;
  const int y0 = seg * a.seg_rows;
  const int y1 = y0 + a.seg_rows < H ? y0 + a.seg_rows : H;
  const int64_t col = inx ? x : 0;
  const int R2 = 2 * r + 1;
  // the plane(s) a value is formed from: one (FP64 or FP32 planes) or two
  // (a product channel; the second factor's plane is read for first
  // moments and the count too, and weighted out)
  const raw_t* pu;
  const raw_t* pv = nullptr;
  double cu = 0.0, cv = 0.0, ku = 1.0, kv = 1.0;
  if constexpr (SRC == BOX_AVGFIELDS) {
    // plane by < C: 1 * G_by; else g~_q * G_c with by = C + q C + c
    const bool ones = by < a.C;
    const int q = ones ? 0 : (by - a.C) / a.C;
    const int c = ones ? by : (by - a.C) % a.C;
    const float* fu = a.guides + (int64_t)q * a.plane;
    const float* fv = a.gout + (int64_t)c * a.plane;
    cu = fu[0];
    ku = ones ? 0.0 : 1.0;
    pu = fu + col;
    pv = fv + col;
  } else if constexpr (PRODUCTS) {
    int u, v;
    const int ch = by - a.count_first;
    const bool ones = ch < 0;  // the pixel count: every factor is 1
    channel_factors(ones ? 0 : ch, a.Q, a.C, &u, &v);
    const bool single = v < 0;  // a first moment: the second factor is 1
    const float* fu = input_plane(a, u);
    const float* fv = single ? fu : input_plane(a, v);
    cu = fu[0];
    cv = fv[0];
    ku = ones ? 0.0 : 1.0;
    kv = ones || single ? 0.0 : 1.0;
    pu = fu + col;
    pv = fv + col;
  } else if constexpr (SRC == BOX_MEAN32) {
    pu = a.srcf + (int64_t)by * a.plane + col;
  } else {  // BOX_SUM64, BOX_MEAN64
    pu = a.src + (int64_t)by * a.plane + col;
  }
  // the window count of this lane's column (BOX_AVGFIELDS)
  const int ncx0 = (x + r < W - 1 ? x + r : W - 1) - (x - r > 0 ? x - r : 0) + 1;
  const int ncx = ncx0 > 0 ? ncx0 : 1;  // lanes right of the image (masked) stay finite
  // value of a loaded row yy: ((u - cu) ku + 1 - ku) ((v - cv) kv + 1 - kv)
  // for products (no branch on the channel kind), u ((v / n) for the
  // averaging products), the plane value otherwise
  auto value = [&](raw_t u, raw_t v, int yy) -> double {
    if constexpr (SRC == BOX_AVGFIELDS) {
      const int ncy = (yy + r < H - 1 ? yy + r : H - 1) - (yy - r > 0 ? yy - r : 0) + 1;
      const double inv_n = 1.0 / (double)(ncy * ncx);
      const double t = ((double)u - cu) * ku + (1.0 - ku);
      return t * ((double)v * inv_n);
    } else if constexpr (PRODUCTS) {
      (void)yy;
      const double t = ((double)u - cu) * ku + (1.0 - ku);
      const double w = ((double)v - cv) * kv + (1.0 - kv);
      return t * w;
    } else {
      (void)v;
      (void)yy;
      return (double)u;
    }
  };
  auto clamp_row = [&](int yy) { return yy < 0 ? 0 : (yy >= H ? H - 1 : yy); };
  // Loads of kRowBatch rows from clamped addresses, unconditional (masked
  // when used), so that they are in flight together; the next batch's loads
  // are issued before the current batch is summed.
  constexpr int kRowBatch = 8;
  auto load_rows = [&](int ybase, raw_t (&u)[kRowBatch], raw_t (&v)[kRowBatch]) {
#pragma unroll
    for (int k = 0; k < kRowBatch; ++k) {
      const int64_t o = (int64_t)clamp_row(ybase + k) * W;
      u[k] = pu[o];
      if constexpr (PRODUCTS) v[k] = pv[o];
    }
  };
  double* dst = SRC == BOX_MEAN32 ? nullptr : a.dst + (int64_t)by * a.plane;  // FP64 out
  const bool owner = inx && tid >= r && tid < kThreads - r;
  // the window of an owner lane: lanes tid - r .. tid + r
  const HWin hw = hwin<WIDE>(tid >= r ? tid - r : 0, r);
  if (tid < 2) rows[tid * (kThreads + 1) + kThreads] = 0.0;  // pads (ordered by the first barrier)
  double v = 0.0;
  {
    // rows y0 - r .. y0 + r; with the ring, row yy goes to slot yy - (y0 - r)
    const int lo = y0 - r, hi = y0 + r;
    for (int yb = lo; yb <= hi; yb += kRowBatch) {
      raw_t tu[kRowBatch], tv[kRowBatch];
      load_rows(yb, tu, tv);
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
        const int yy = yb + u;
        const double m = (inx && yy >= 0 && yy < H) ? value(tu[u], tv[u], yy) : 0.0;
        if (yy <= hi) {
          v += m;
          if constexpr (RING) ring[(yy - lo) * kThreads] = m;
        }
      }
    }
  }
  // At step y > y0 the row leaving the window, y - r - 1, sits in slot
  // (y - y0 - 1) mod (2r + 1), the slot the entering row y + r takes over.
  int slot = 0;
  raw_t eu[kRowBatch], ev[kRowBatch], lu[kRowBatch], lv[kRowBatch];
  load_rows(y0 + r, eu, ev);
  if constexpr (!RING) load_rows(y0 - r - 1, lu, lv);
  for (int yc = y0; yc < y1; yc += kRowBatch) {
    raw_t nu[kRowBatch], nv[kRowBatch], mu[kRowBatch], mv[kRowBatch];
    load_rows(yc + kRowBatch + r, nu, nv);
    if constexpr (!RING) load_rows(yc + kRowBatch - r - 1, mu, mv);
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {
      const int y = yc + u;
      if (y >= y1) break;  // uniform across the workgroup
      if (y > y0) {
        const double e = (inx && y + r < H) ? value(eu[u], ev[u], y + r) : 0.0;
        double l;
        if constexpr (RING) {
          double* rs = ring + slot * kThreads;
          l = *rs;
          *rs = e;
          slot = slot + 1 == R2 ? 0 : slot + 1;
        } else {
          l = (inx && y - r - 1 >= 0) ? value(lu[u], lv[u], y - r - 1) : 0.0;
        }
        v += e - l;
      }
      // alternate prefix rows: one barrier per row orders this row's writes
      // before its reads, and the reads of two rows back before these writes
      double* P = rows + ((y - y0) & 1) * (kThreads + 1);
      P[tid] = seg_prefix<WIDE>(v);
      __syncthreads();
      if (owner) {
        const double s = hwin_sum(P, hw);
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
#pragma unroll
    for (int k = 0; k < kRowBatch; ++k) {
      eu[k] = nu[k];
      if constexpr (PRODUCTS) ev[k] = nv[k];
      if constexpr (!RING) {
        lu[k] = mu[k];
        if constexpr (PRODUCTS) lv[k] = mv[k];
      }
    }
  }
}

// box_tile with the ring when the arguments ask for it.
template <int SRC, bool WIDE>
__device__ __forceinline__ void box_tile_any(const AdjBoxArgs& a, const int bx, const int by) {
  if (a.ring)
    box_tile<SRC, WIDE, true>(a, bx, by);
  else
    box_tile<SRC, WIDE, false>(a, bx, by);
}

}  // namespace flr
