// Device code of the FLR path for gfx950, templated on the guide count Q and
// the channel count C so that every per-pixel array lives in registers.
//
// Window sums (Sec. 3.2) are separable: a workgroup owns a strip of
// kThreads consecutive columns and walks down a segment of rows. Each lane
// keeps the vertical running sums of all moment channels of its column in
// registers (add the row entering the window, subtract the row leaving it,
// products re-formed from the re-read inputs instead of being stored). Each
// row of vertical sums is then staged through LDS, where lanes take
// (channel, column-chunk) tasks and slide the horizontal window along the
// chunk. The lane that owns a column reads back its full window sums, forms
// central moments and solves the regularised system with a Cholesky
// factorisation held in registers.
//
// Conditioning: the guides are shifted by a per-workgroup anchor (their
// value at one pixel of the tile) before products are formed; central
// moments are invariant to the shift. Coefficients are kept relative to the
// same anchor (b~ = nu - a^T mu~) so that averaging and reconstruction never
// form the large, cancelling original-unit intercepts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "flr_launch.hpp"

namespace flr {

template <int Q, int C>
struct Dims {
  static constexpr int F = Q + 1;
  static constexpr int NP = Q * (Q + 1) / 2;  // guide x guide products (upper triangle)
  static constexpr int NQC = Q * C;           // guide x channel products
  static constexpr int NS = Q + C + NP + NQC; // summed channels (n is analytic)
  static constexpr int FC = F * C;            // coefficients per pixel
  static constexpr int MG = group_size(NS, sizeof(sum_t));   // moment rows per LDS group
  static constexpr int AG = group_size(FC, sizeof(solve_t)); // coefficient rows per LDS group
};

// Index of (p, q), p <= q, in a row-major packed upper triangle.
template <int Q>
__host__ __device__ constexpr int tri(int p, int q) {
  return p * Q - p * (p - 1) / 2 + (q - p);
}

__device__ __forceinline__ int win_count(int i, int n, int r) {
  const int lo = i - r < 0 ? 0 : i - r;
  const int hi = i + r > n - 1 ? n - 1 : i + r;
  return hi - lo + 1;
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float rsqrt_t(float x) { return rsqrtf(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return 1.0 / sqrt(x); }

// max(x, 0) that lets NaN through.
template <typename T>
__device__ __forceinline__ T clamp_nonneg(T x) {
  return x < T(0) ? T(0) : x;
}

// ---------------------------------------------------------------------------
// Regularised system: on entry Hm holds the guide covariance (upper
// triangle); mu_o are the window means in original units.
template <int Q, typename T>
__device__ __forceinline__ void regularise(T (&Hm)[Q * (Q + 1) / 2], const T (&mu_o)[Q], T eps,
                                           T eps_mul, int mode) {
#pragma unroll
  for (int q = 0; q < Q; ++q) Hm[tri<Q>(q, q)] = clamp_nonneg(Hm[tri<Q>(q, q)]);
  if (mode == 0) {  // ridge: W + eps I
#pragma unroll
    for (int q = 0; q < Q; ++q) Hm[tri<Q>(q, q)] += eps;
  } else {  // Appendix: W^ = W + eps' (mu mu^T + diag(mu o mu)) + eps I; H = W^ + eps diag(W^)
#pragma unroll
    for (int p = 0; p < Q; ++p) {
#pragma unroll
      for (int q = p; q < Q; ++q) {
        const T mm = mu_o[p] * mu_o[q];
        Hm[tri<Q>(p, q)] = fma_t(eps_mul, p == q ? T(2) * mm : mm, Hm[tri<Q>(p, q)]);
      }
    }
    const T s = T(1) + eps;
#pragma unroll
    for (int q = 0; q < Q; ++q) Hm[tri<Q>(q, q)] = (Hm[tri<Q>(q, q)] + eps) * s;
  }
}

// Solve H X = R for C right-hand sides (R is [Q][C] row-major, overwritten
// by X). H = U^T U with U upper triangular, built in place in Hm; only the
// reciprocals of the diagonal of U are kept.
template <int Q, int C, typename T>
__device__ __forceinline__ void chol_solve(T (&Hm)[Q * (Q + 1) / 2], T (&R)[Q * C]) {
  T inv[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    T d = Hm[tri<Q>(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) d = fma_t(-Hm[tri<Q>(k, j)], Hm[tri<Q>(k, j)], d);
    if (d < T(1e-30)) d = T(1e-30);
    const T ij = rsqrt_t(d);
    inv[j] = ij;
#pragma unroll
    for (int i = j + 1; i < Q; ++i) {
      T s = Hm[tri<Q>(j, i)];
#pragma unroll
      for (int k = 0; k < j; ++k) s = fma_t(-Hm[tri<Q>(k, j)], Hm[tri<Q>(k, i)], s);
      Hm[tri<Q>(j, i)] = s * ij;
    }
  }
  // U^T z = R
#pragma unroll
  for (int j = 0; j < Q; ++j) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      T s = R[j * C + c];
#pragma unroll
      for (int k = 0; k < j; ++k) s = fma_t(-Hm[tri<Q>(k, j)], R[k * C + c], s);
      R[j * C + c] = s * inv[j];
    }
  }
  // U x = z
#pragma unroll
  for (int j = Q - 1; j >= 0; --j) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      T s = R[j * C + c];
#pragma unroll
      for (int k = j + 1; k < Q; ++k) s = fma_t(-Hm[tri<Q>(j, k)], R[k * C + c], s);
      R[j * C + c] = s * inv[j];
    }
  }
}

// ---------------------------------------------------------------------------
// Horizontal window sums of `rows` LDS rows: dst[m][j] = sum_{k=0..2r}
// src[m][j+k] for j < nout. Tasks are (row, chunk of `chunk` outputs); the
// first output of a chunk is a direct sum, the rest slide.
template <typename E>
__device__ __forceinline__ void hbox(const E* __restrict__ src, E* __restrict__ dst, int rows,
                                     int nout, int r, int chunk) {
  const int nch = (nout + chunk - 1) / chunk;
  const int ntask = rows * nch;
  for (int t = threadIdx.x; t < ntask; t += kThreads) {
    const int m = t % rows;
    const int ch = t / rows;
    const E* s = src + m * kLdsStride;
    E* d = dst + m * kLdsStride;
    const int j0 = ch * chunk;
    const int j1 = min(j0 + chunk, nout);
    E acc = E(0);
    for (int k = 0; k <= 2 * r; ++k) acc += s[j0 + k];
    d[j0] = acc;
    for (int jj = j0 + 1; jj < j1; ++jj) {
      acc += s[jj + 2 * r] - s[jj - 1];
      d[jj] = acc;
    }
  }
}

// Guides (shifted by the anchor) and noisy values of one pixel; zeros when
// the pixel is outside the image so that it contributes nothing.
template <int Q, int C>
__device__ __forceinline__ void load_px(const LaunchArgs& a, int64_t pl, int64_t off, bool ok,
                                        const float (&cg)[Q], sum_t (&g)[Q], sum_t (&y)[C]) {
  if (ok) {
#pragma unroll
    for (int q = 0; q < Q; ++q) g[q] = (sum_t)a.guides[q * pl + off] - (sum_t)cg[q];
#pragma unroll
    for (int c = 0; c < C; ++c) y[c] = (sum_t)a.noisy[c * pl + off];
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) g[q] = sum_t(0);
#pragma unroll
    for (int c = 0; c < C; ++c) y[c] = sum_t(0);
  }
}

// Channel order: sum g[Q] | sum y[C] | sum g_p g_q (p<=q) | sum g_q y_c.
// V += products of the entering pixel (ga, ya) - those of the leaving one.
template <int Q, int C>
__device__ __forceinline__ void vupdate(sum_t (&V)[num_sums(Q, C)], const sum_t (&ga)[Q],
                                        const sum_t (&ya)[C], const sum_t (&gs)[Q],
                                        const sum_t (&ys)[C]) {
#pragma unroll
  for (int q = 0; q < Q; ++q) V[q] += ga[q] - gs[q];
#pragma unroll
  for (int c = 0; c < C; ++c) V[Q + c] += ya[c] - ys[c];
  int k = Q + C;
#pragma unroll
  for (int p = 0; p < Q; ++p) {
#pragma unroll
    for (int q = p; q < Q; ++q) {
      V[k] = fma_t(-gs[p], gs[q], fma_t(ga[p], ga[q], V[k]));
      ++k;
    }
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      V[k] = fma_t(-gs[q], ys[c], fma_t(ga[q], ya[c], V[k]));
      ++k;
    }
  }
}

// Position of channel m of the upper-triangle block: row p, column q.
template <int Q>
__host__ __device__ constexpr int tri_row(int k) {
  int p = 0;
  while (k >= Q - p) {
    k -= Q - p;
    ++p;
  }
  return p;
}
template <int Q>
__host__ __device__ constexpr int tri_col(int k) {
  int p = 0;
  while (k >= Q - p) {
    k -= Q - p;
    ++p;
  }
  return p + k;
}

// Fold window sum v of channel m (order: sum g | sum y | sum g_p g_q |
// sum g_q y_c, shifted guides) into the central moments: mu~, nu, the
// guide covariance Hm and the guide/channel covariance R. Channels arrive in
// increasing m, so the means are complete before any covariance needs them.
template <int Q, int C, typename T>
__device__ __forceinline__ void centre_channel(int m, T v, T inv_n, T (&mu)[Q], T (&nu)[C],
                                               T (&Hm)[Q * (Q + 1) / 2], T (&R)[Q * C]) {
  constexpr int NP = Q * (Q + 1) / 2;
  if (m < Q) {
    mu[m] = v * inv_n;
  } else if (m < Q + C) {
    nu[m - Q] = v * inv_n;
  } else if (m < Q + C + NP) {
    const int k = m - Q - C;
    Hm[k] = fma_t(v, inv_n, -mu[tri_row<Q>(k)] * mu[tri_col<Q>(k)]);
  } else {
    const int k = m - Q - C - NP;
    R[k] = fma_t(v, inv_n, -mu[k / C] * nu[k % C]);
  }
}

// Horizontal sums of the F*C coefficient rows held in LDS (t0, written by
// the caller in groups via `fill`), and the reconstruction
//   out_c = (sum b~_c + sum_q g~_q sum a_qc) / n   for output lane `o`.
// `fill(f0, gn, t0)` writes coefficient rows f0..f0+gn-1 into t0.
template <int Q, int C, typename Fill>
__device__ __forceinline__ void average_and_reconstruct(solve_t* t0, solve_t* t1, int nout, int r,
                                                        int chunk, bool active,
                                                        const solve_t (&gq)[Q], solve_t inv_n,
                                                        float* out_c0, int64_t pl, Fill fill) {
  using D = Dims<Q, C>;
  constexpr int FC = D::FC;
  constexpr int AG = D::AG;
  solve_t acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = solve_t(0);
#pragma unroll
  for (int f0 = 0; f0 < FC; f0 += AG) {
    const int gn = FC - f0 < AG ? FC - f0 : AG;
    __syncthreads();
    fill(f0, gn, t0);
    __syncthreads();
    hbox(t0, t1, gn, nout, r, chunk);
    __syncthreads();
    if (active) {
#pragma unroll
      for (int k = 0; k < gn; ++k) {
        const int f = f0 + k;
        const solve_t v = t1[k * kLdsStride + threadIdx.x];
        if (f < C) {
          acc[f] += v;
        } else {
          const int q = f / C - 1;
          const int c = f % C;
          acc[c] = fma_t(gq[q], v, acc[c]);
        }
      }
    }
  }
  if (active) {
#pragma unroll
    for (int c = 0; c < C; ++c) out_c0[c * pl] = (float)(acc[c] * inv_n);
  }
}

enum WalkMode : int { W_MOMENTS = 0, W_FUSED0 = 1, W_FUSED1 = 2 };

// ---------------------------------------------------------------------------
// The walker. MODE selects what happens with the window moments of each
// coefficient position:
//   W_MOMENTS  write the moment planes (central, or raw sums with a.raw);
//   W_FUSED0   solve and reconstruct at the same pixel;
//   W_FUSED1   solve, push the coefficients through a per-workgroup ring of
//              2r+1 rows (global workspace) to form vertical window sums,
//              stage those through LDS for the horizontal sums, and
//              reconstruct with the averaged coefficients. The segment is
//              extended by r coefficient rows above and below and the strip
//              by r columns each side, so no data crosses workgroups.
template <int Q, int C, int MODE>
__global__ void __launch_bounds__(kThreads, 1) walk_kernel(LaunchArgs a) {
  using D = Dims<Q, C>;
  using T = solve_t;
  constexpr int NS = D::NS;
  constexpr int FC = D::FC;
  constexpr int NP = D::NP;
  constexpr int MG = D::MG;
  constexpr size_t BYTES_M = (size_t)MG * sizeof(sum_t);
  constexpr size_t BYTES_A = (size_t)D::AG * sizeof(T);
  constexpr size_t HALF = (BYTES_M > BYTES_A ? BYTES_M : BYTES_A) * kLdsStride;
  extern __shared__ float lds[];
  sum_t* S0 = reinterpret_cast<sum_t*>(lds);
  sum_t* S1 = reinterpret_cast<sum_t*>(reinterpret_cast<char*>(lds) + HALF);
  T* T0 = reinterpret_cast<T*>(lds);
  T* T1 = reinterpret_cast<T*>(reinterpret_cast<char*>(lds) + HALF);

  const int tid = threadIdx.x;
  const int r = a.r;
  const int H = a.H;
  const int W = a.W;
  const int64_t pl = (int64_t)H * W;
  const int hc = MODE == W_FUSED1 ? r : 0;
  const int ncoef = kThreads - 2 * r;
  const int tout = ncoef - 2 * hc;
  const int sx = blockIdx.x % a.tiles_x;
  const int sy = blockIdx.x / a.tiles_x;
  const int X0 = sx * tout;
  const int Y0 = sy * a.seg_rows;
  const int Y1 = min(Y0 + a.seg_rows, H);
  const int xi = X0 - hc - r + tid;  // input column of this lane
  const bool xin = xi >= 0 && xi < W;
  const int xc = X0 - hc + tid;      // coefficient column of this lane (tid < ncoef)
  const bool cvalid = tid < ncoef && xc >= 0 && xc < W;

  float cg[Q];
  {
    const int yr = min(max((Y0 + Y1) / 2, 0), H - 1);
    const int xr = min(max(X0 + tout / 2, 0), W - 1);
#pragma unroll
    for (int q = 0; q < Q; ++q) cg[q] = a.raw ? 0.f : a.guides[q * pl + (int64_t)yr * W + xr];
  }

  sum_t V[NS];
#pragma unroll
  for (int m = 0; m < NS; ++m) V[m] = sum_t(0);

  const int ym0 = Y0 - hc;
  const int ym1 = Y1 + hc;
  {
    sum_t zg[Q], zy[C];
#pragma unroll
    for (int q = 0; q < Q; ++q) zg[q] = sum_t(0);
#pragma unroll
    for (int c = 0; c < C; ++c) zy[c] = sum_t(0);
    for (int yy = ym0 - r; yy < ym0 + r; ++yy) {
      if (yy < 0 || yy >= H) continue;
      sum_t g[Q], y[C];
      load_px<Q, C>(a, pl, (int64_t)yy * W + xi, xin, cg, g, y);
      vupdate<Q, C>(V, g, y, zg, zy);
    }
  }

  constexpr int NVA = MODE == W_FUSED1 ? FC : 1;
  T Va[NVA];
#pragma unroll
  for (int f = 0; f < NVA; ++f) Va[f] = T(0);
  ring_t* ring =
      reinterpret_cast<ring_t*>(a.ring) + (size_t)blockIdx.x * (size_t)(2 * r + 1) * FC * kThreads + tid;

  for (int ym = ym0; ym < ym1; ++ym) {
    {
      const int ya = ym + r;
      const int ys = ym - r - 1;
      const bool oka = ya >= 0 && ya < H;
      const bool oks = ym > ym0 && ys >= 0 && ys < H;
      sum_t ga[Q], yA[C], gs[Q], yS[C];
      load_px<Q, C>(a, pl, (int64_t)ya * W + xi, xin && oka, cg, ga, yA);
      load_px<Q, C>(a, pl, (int64_t)ys * W + xi, xin && oks, cg, gs, yS);
      vupdate<Q, C>(V, ga, yA, gs, yS);
    }
    const bool row_in = ym >= 0 && ym < H;

    T cv[NVA];
#pragma unroll
    for (int f = 0; f < NVA; ++f) cv[f] = T(0);

    if (row_in) {
      const int64_t off = (int64_t)ym * W + xc;
      const int ni = cvalid ? win_count(ym, H, r) * win_count(xc, W, r) : 1;
      const T inv_n = T(1) / (T)ni;
      T mu[Q], nu[C], Hm[NP], R[Q * C];
#pragma unroll
      for (int g0 = 0; g0 < NS; g0 += MG) {
        const int gn = NS - g0 < MG ? NS - g0 : MG;
        __syncthreads();
#pragma unroll
        for (int m = 0; m < gn; ++m) S0[m * kLdsStride + tid] = V[g0 + m];
        __syncthreads();
        hbox(S0, S1, gn, ncoef, r, a.hchunk_m);
        __syncthreads();
        if (cvalid) {
#pragma unroll
          for (int m = 0; m < gn; ++m) {
            const sum_t v = S1[m * kLdsStride + tid];
            if (MODE == W_MOMENTS && a.raw)
              a.out[(1 + g0 + m) * pl + off] = (float)v;
            else
              centre_channel<Q, C, T>(g0 + m, (T)v, inv_n, mu, nu, Hm, R);
          }
        }
      }
      if (cvalid) {
        if (MODE == W_MOMENTS) {
          a.out[off] = (float)ni;
          if (!a.raw) {
#pragma unroll
            for (int q = 0; q < Q; ++q) a.out[(1 + q) * pl + off] = (float)(mu[q] + (T)cg[q]);
#pragma unroll
            for (int c = 0; c < C; ++c) a.out[(1 + Q + c) * pl + off] = (float)nu[c];
#pragma unroll
            for (int k = 0; k < NP; ++k) a.out[(1 + Q + C + k) * pl + off] = (float)Hm[k];
#pragma unroll
            for (int k = 0; k < Q * C; ++k) a.out[(1 + Q + C + NP + k) * pl + off] = (float)R[k];
          }
        } else {
          T mu_o[Q];
#pragma unroll
          for (int q = 0; q < Q; ++q) mu_o[q] = mu[q] + (T)cg[q];
          regularise<Q, T>(Hm, mu_o, (T)a.eps, (T)a.eps_mul, a.reg_mode);
          chol_solve<Q, C, T>(Hm, R);
          if (MODE == W_FUSED0) {
            T gp[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) gp[q] = ((T)a.guides[q * pl + off] - (T)cg[q]) - mu[q];
#pragma unroll
            for (int c = 0; c < C; ++c) {
              T acc = nu[c];
#pragma unroll
              for (int q = 0; q < Q; ++q) acc = fma_t(gp[q], R[q * C + c], acc);
              a.out[c * pl + off] = (float)acc;
            }
          } else {
            // coefficients relative to the anchor: b~ = nu - a^T mu~
#pragma unroll
            for (int c = 0; c < C; ++c) {
              T b = nu[c];
#pragma unroll
              for (int q = 0; q < Q; ++q) b = fma_t(-R[q * C + c], mu[q], b);
              cv[c] = b;
            }
#pragma unroll
            for (int k = 0; k < Q * C; ++k) cv[C + k] = R[k];
          }
        }
      }
    }

    if (MODE == W_FUSED1) {
      // vertical window sums of the coefficients through the ring
      if (tid < ncoef) {
        const int slot = (ym - ym0) % (2 * r + 1);
        ring_t* rs = ring + (size_t)slot * FC * kThreads;
        const int yold = ym - 2 * r - 1;
        const bool okold = yold >= ym0 && yold >= 0 && yold < H;
#pragma unroll
        for (int f = 0; f < FC; ++f) {
          // the ring holds the stored (rounded) values, so add those too
          const ring_t nw = (ring_t)cv[f];
          const T old = okold ? (T)rs[f * kThreads] : T(0);
          Va[f] += (T)nw - old;
        }
        if (row_in) {
#pragma unroll
          for (int f = 0; f < FC; ++f) rs[f * kThreads] = (ring_t)cv[f];
        }
      }
      const int yo = ym - r;
      if (yo >= Y0 && yo < Y1) {
        const int xo = X0 + tid;
        const bool active = tid < tout && xo < W;
        const int64_t off = (int64_t)yo * W + (active ? xo : 0);
        T gq[Q];
        T inv = T(0);
        if (active) {
#pragma unroll
          for (int q = 0; q < Q; ++q) gq[q] = ((T)a.guides[q * pl + off] - (T)cg[q]);
          inv = T(1) / (T)(win_count(yo, H, r) * win_count(xo, W, r));
        } else {
#pragma unroll
          for (int q = 0; q < Q; ++q) gq[q] = T(0);
        }
        average_and_reconstruct<Q, C>(
            T0, T1, tout, r, a.hchunk_a, active, gq, inv, a.out + off, pl,
            [&](int f0, int gn, T* dst) {
              if (tid < ncoef) {
#pragma unroll
                for (int k = 0; k < gn; ++k) dst[k * kLdsStride + tid] = Va[f0 + k];
              }
            });
      }
    }
  }
}

// ---------------------------------------------------------------------------
// flr_solve: one lane per pixel, central-moment planes -> coefficient planes.
template <int Q, int C>
__global__ void __launch_bounds__(256) solve_kernel(LaunchArgs a) {
  using T = solve_t;
  constexpr int NP = Dims<Q, C>::NP;
  const int64_t pl = (int64_t)a.H * a.W;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= pl) return;
  const float* m = a.planes + idx;
  T mu[Q], nu[C], Hm[NP], R[Q * C];
#pragma unroll
  for (int q = 0; q < Q; ++q) mu[q] = m[(1 + q) * pl];
#pragma unroll
  for (int c = 0; c < C; ++c) nu[c] = m[(1 + Q + c) * pl];
#pragma unroll
  for (int k = 0; k < NP; ++k) Hm[k] = m[(1 + Q + C + k) * pl];
#pragma unroll
  for (int k = 0; k < Q * C; ++k) R[k] = m[(1 + Q + C + NP + k) * pl];
  regularise<Q, T>(Hm, mu, (T)a.eps, (T)a.eps_mul, a.reg_mode);
  chol_solve<Q, C, T>(Hm, R);
  float* o = a.out + idx;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    T b = nu[c];
#pragma unroll
    for (int q = 0; q < Q; ++q) b = fma_t(-R[q * C + c], mu[q], b);
    o[c * pl] = (float)b;
  }
#pragma unroll
  for (int k = 0; k < Q * C; ++k) o[(C + k) * pl] = (float)R[k];
}

// flr_apply without averaging: out_c = b_c + sum_q g_q a_qc per pixel.
template <int Q, int C>
__global__ void __launch_bounds__(256) apply_point_kernel(LaunchArgs a) {
  using T = solve_t;
  const int64_t pl = (int64_t)a.H * a.W;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= pl) return;
  T g[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) g[q] = a.guides[q * pl + idx];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    T acc = a.planes[c * pl + idx];
#pragma unroll
    for (int q = 0; q < Q; ++q) acc = fma_t(g[q], (T)a.planes[((1 + q) * C + c) * pl + idx], acc);
    a.out[c * pl + idx] = (float)acc;
  }
}

// flr_apply with averaging: a walker over coefficient planes. Lanes own
// coefficient columns [X0 - r, X0 - r + kThreads) and keep vertical window
// sums of all F*C coefficient planes; horizontal sums go through LDS.
template <int Q, int C>
__global__ void __launch_bounds__(kThreads, 1) apply_avg_kernel(LaunchArgs a) {
  using T = solve_t;
  constexpr int FC = Dims<Q, C>::FC;
  constexpr size_t HALF = (size_t)Dims<Q, C>::AG * sizeof(T) * kLdsStride;
  extern __shared__ float lds[];
  T* T0 = reinterpret_cast<T*>(lds);
  T* T1 = reinterpret_cast<T*>(reinterpret_cast<char*>(lds) + HALF);
  const int tid = threadIdx.x;
  const int r = a.r;
  const int H = a.H;
  const int W = a.W;
  const int64_t pl = (int64_t)H * W;
  const int tout = kThreads - 2 * r;
  const int sx = blockIdx.x % a.tiles_x;
  const int sy = blockIdx.x / a.tiles_x;
  const int X0 = sx * tout;
  const int Y0 = sy * a.seg_rows;
  const int Y1 = min(Y0 + a.seg_rows, H);
  const int xcol = X0 - r + tid;
  const bool xin = xcol >= 0 && xcol < W;

  T Va[FC];
#pragma unroll
  for (int f = 0; f < FC; ++f) Va[f] = T(0);
  for (int yy = Y0 - r; yy < Y0 + r; ++yy) {
    if (yy < 0 || yy >= H || !xin) continue;
    const int64_t off = (int64_t)yy * W + xcol;
#pragma unroll
    for (int f = 0; f < FC; ++f) Va[f] += (T)a.planes[f * pl + off];
  }
  for (int yo = Y0; yo < Y1; ++yo) {
    const int ya = yo + r;
    const int ys = yo - r - 1;
    const bool oka = xin && ya < H;
    const bool oks = xin && yo > Y0 && ys >= 0;
    const int64_t offa = (int64_t)ya * W + xcol;
    const int64_t offs = (int64_t)ys * W + xcol;
#pragma unroll
    for (int f = 0; f < FC; ++f) {
      const T add = oka ? (T)a.planes[f * pl + offa] : T(0);
      const T sub = oks ? (T)a.planes[f * pl + offs] : T(0);
      Va[f] += add - sub;
    }
    const int xo = X0 + tid;
    const bool active = tid < tout && xo < W;
    const int64_t off = (int64_t)yo * W + (active ? xo : 0);
    T gq[Q];
    T inv = T(0);
    if (active) {
#pragma unroll
      for (int q = 0; q < Q; ++q) gq[q] = (T)a.guides[q * pl + off];
      inv = T(1) / (T)(win_count(yo, H, r) * win_count(xo, W, r));
    } else {
#pragma unroll
      for (int q = 0; q < Q; ++q) gq[q] = T(0);
    }
    average_and_reconstruct<Q, C>(T0, T1, tout, r, a.hchunk_a, active, gq, inv, a.out + off, pl,
                                  [&](int f0, int gn, T* dst) {
#pragma unroll
                                    for (int k = 0; k < gn; ++k)
                                      dst[k * kLdsStride + tid] = Va[f0 + k];
                                  });
  }
}

// ---------------------------------------------------------------------------
// Host-side launch of one kernel kind for a fixed (Q, C).
template <typename K>
static hipError_t launch_with_lds(K kernel, int blocks, size_t lds, const LaunchArgs& a,
                                  hipStream_t s) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kernel, dim3(blocks), dim3(kThreads), lds, s, a);
  return hipGetLastError();
}

template <int Q, int C>
hipError_t launch_qc(int kind, const LaunchArgs& a, hipStream_t s) {
  const int64_t pl = (int64_t)a.H * a.W;
  const int pblocks = (int)((pl + 255) / 256);
  const int wblocks = a.tiles_x * a.n_seg;
  switch (kind) {
    case K_MOMENTS:
      return launch_with_lds(walk_kernel<Q, C, W_MOMENTS>, wblocks, walk_lds_bytes(kind, Q, C), a, s);
    case K_FUSED0:
      return launch_with_lds(walk_kernel<Q, C, W_FUSED0>, wblocks, walk_lds_bytes(kind, Q, C), a, s);
    case K_FUSED1:
      return launch_with_lds(walk_kernel<Q, C, W_FUSED1>, wblocks, walk_lds_bytes(kind, Q, C), a, s);
    case K_APPLY_AVG:
      return launch_with_lds(apply_avg_kernel<Q, C>, wblocks, walk_lds_bytes(kind, Q, C), a, s);
    case K_SOLVE:
      hipLaunchKernelGGL((solve_kernel<Q, C>), dim3(pblocks), dim3(256), 0, s, a);
      return hipGetLastError();
    case K_APPLY_POINT:
      hipLaunchKernelGGL((apply_point_kernel<Q, C>), dim3(pblocks), dim3(256), 0, s, a);
      return hipGetLastError();
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace flr

#define FLR_DEFINE_Q(q)                                                                 \
  namespace flr {                                                                       \
  hipError_t launch_q##q(int C, int kind, const LaunchArgs& a, hipStream_t s) {         \
    switch (C) {                                                                        \
      case 1: return launch_qc<q, 1>(kind, a, s);                                       \
      case 2: return launch_qc<q, 2>(kind, a, s);                                       \
      case 3: return launch_qc<q, 3>(kind, a, s);                                       \
      case 4: return launch_qc<q, 4>(kind, a, s);                                       \
      default: return hipErrorInvalidValue;                                             \
    }                                                                                   \
  }                                                                                     \
  }
