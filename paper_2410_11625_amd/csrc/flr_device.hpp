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

#include <type_traits>

#include "flr.h"
#include "flr_launch.hpp"
#include "flr_prefix.hpp"

namespace flr {

template <int Q, int C>
struct Dims {
  static constexpr int F = Q + 1;
  static constexpr int NP = Q * (Q + 1) / 2;  // guide x guide products (upper triangle)
  static constexpr int NQC = Q * C;           // guide x channel products
  static constexpr int NS = Q + C + NP + NQC; // summed channels (n is analytic)
  static constexpr int FC = F * C;            // coefficients per pixel
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
// FP64 1/sqrt(x): the FP32 hardware estimate (about 2^-23 relative) refined
// by one Newton step (error squared, about 2^-46, far below what the FP32
// inputs carry); outside the FP32 range, plain 1/sqrt.
__device__ __forceinline__ double rsqrt_t(double x) {
  if (!(x > 1e-36 && x < 1e36)) return 1.0 / sqrt(x);
  double y = (double)rsqrtf((float)x);
  const double e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}
// 1/n for a window count n >= 1, refined the same way.
__device__ __forceinline__ float recip_count(int n, float) { return 1.f / (float)n; }
__device__ __forceinline__ double recip_count(int n, double) {
  const double d = (double)n;
  const double y = (double)(1.f / (float)n);
  return fma(y, fma(-d, y, 1.0), y);
}

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

// The regularisers of a launch: its arguments, or the device pair (eps,
// eps_mul) when the caller keeps them on the device.
__device__ __forceinline__ float arg_eps(const LaunchArgs& a) {
  return a.eps_dev ? a.eps_dev[0] : a.eps;
}
__device__ __forceinline__ float arg_eps_mul(const LaunchArgs& a) {
  return a.eps_dev ? a.eps_dev[1] : a.eps_mul;
}

// f(std::integral_constant<int, I>) for I = B .. E-1: loop bodies with
// compile-time indices, whatever the trip count (the compiler otherwise
// keeps short inner loops of the larger systems as loops over arrays in
// scratch memory).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Solve H X = R for C right-hand sides (R is [Q][C] row-major, overwritten
// by X). H = U^T U with U upper triangular, built in place in Hm; only the
// reciprocals of the diagonal of U are kept.
template <int Q, int C, typename T>
__device__ __forceinline__ void chol_solve(T (&Hm)[Q * (Q + 1) / 2], T (&R)[Q * C]) {
  T inv[Q];
  static_for<0, Q>([&](auto J) {
    constexpr int j = decltype(J)::value;
    T d = Hm[tri<Q>(j, j)];
    static_for<0, j>([&](auto K) {
      constexpr int k = decltype(K)::value;
      d = fma_t(-Hm[tri<Q>(k, j)], Hm[tri<Q>(k, j)], d);
    });
    if (d < T(1e-30)) d = T(1e-30);
    const T ij = rsqrt_t(d);
    inv[j] = ij;
    static_for<j + 1, Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      T s = Hm[tri<Q>(j, i)];
      static_for<0, j>([&](auto K) {
        constexpr int k = decltype(K)::value;
        s = fma_t(-Hm[tri<Q>(k, j)], Hm[tri<Q>(k, i)], s);
      });
      Hm[tri<Q>(j, i)] = s * ij;
    });
  });
  // U^T z = R
  static_for<0, Q>([&](auto J) {
    constexpr int j = decltype(J)::value;
    static_for<0, C>([&](auto Cc) {
      constexpr int c = decltype(Cc)::value;
      T s = R[j * C + c];
      static_for<0, j>([&](auto K) {
        constexpr int k = decltype(K)::value;
        s = fma_t(-Hm[tri<Q>(k, j)], R[k * C + c], s);
      });
      R[j * C + c] = s * inv[j];
    });
  });
  // U x = z
  static_for<0, Q>([&](auto JJ) {
    constexpr int j = Q - 1 - decltype(JJ)::value;
    static_for<0, C>([&](auto Cc) {
      constexpr int c = decltype(Cc)::value;
      T s = R[j * C + c];
      static_for<j + 1, Q>([&](auto K) {
        constexpr int k = decltype(K)::value;
        s = fma_t(-Hm[tri<Q>(j, k)], R[k * C + c], s);
      });
      R[j * C + c] = s * inv[j];
    });
  });
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
  const int w = 2 * r + 1;
  // Each thread runs two tasks side by side, and issues the loads of four
  // outputs of both at once, so that independent LDS reads overlap.
  for (int t0 = threadIdx.x; t0 < ntask; t0 += 2 * kThreads) {
    const int t1 = t0 + kThreads;
    const int m0 = t0 % rows, j00 = (t0 / rows) * chunk;
    const int n0 = min(chunk, nout - j00);
    const int m1 = t1 < ntask ? t1 % rows : m0;
    const int j01 = t1 < ntask ? (t1 / rows) * chunk : j00;
    const int n1 = t1 < ntask ? min(chunk, nout - j01) : 0;
    const E* s0 = src + m0 * kLdsStride + j00;
    const E* s1 = src + m1 * kLdsStride + j01;
    E* d0 = dst + m0 * kLdsStride + j00;
    E* d1 = dst + m1 * kLdsStride + j01;
    E a0 = E(0), b0 = E(0), c0 = E(0), e0 = E(0);
    E a1 = E(0), b1 = E(0), c1 = E(0), e1 = E(0);
    int k = 0;
    for (; k + 4 <= w; k += 4) {
      a0 += s0[k];
      b0 += s0[k + 1];
      c0 += s0[k + 2];
      e0 += s0[k + 3];
      a1 += s1[k];
      b1 += s1[k + 1];
      c1 += s1[k + 2];
      e1 += s1[k + 3];
    }
    for (; k < w; ++k) {
      a0 += s0[k];
      a1 += s1[k];
    }
    E acc0 = (a0 + b0) + (c0 + e0), acc1 = (a1 + b1) + (c1 + e1);
    d0[0] = acc0;
    if (n1 > 0) d1[0] = acc1;
    const E* x0 = s0 + 2 * r;
    const E* x1 = s1 + 2 * r;
    const int n = min(n0, n1);
    int j = 1;
    for (; j + 4 <= n; j += 4) {
      const E p0 = x0[j], p1 = x0[j + 1], p2 = x0[j + 2], p3 = x0[j + 3];
      const E q0 = s0[j - 1], q1 = s0[j], q2 = s0[j + 1], q3 = s0[j + 2];
      const E u0 = x1[j], u1 = x1[j + 1], u2 = x1[j + 2], u3 = x1[j + 3];
      const E v0 = s1[j - 1], v1 = s1[j], v2 = s1[j + 1], v3 = s1[j + 2];
      acc0 += p0 - q0;
      acc1 += u0 - v0;
      d0[j] = acc0;
      d1[j] = acc1;
      acc0 += p1 - q1;
      acc1 += u1 - v1;
      d0[j + 1] = acc0;
      d1[j + 1] = acc1;
      acc0 += p2 - q2;
      acc1 += u2 - v2;
      d0[j + 2] = acc0;
      d1[j + 2] = acc1;
      acc0 += p3 - q3;
      acc1 += u3 - v3;
      d0[j + 3] = acc0;
      d1[j + 3] = acc1;
    }
    for (int jj = j; jj < n0; ++jj) {
      acc0 += x0[jj] - s0[jj - 1];
      d0[jj] = acc0;
    }
    for (int jj = (n1 > 0 ? j : n1); jj < n1; ++jj) {
      acc1 += x1[jj] - s1[jj - 1];
      d1[jj] = acc1;
    }
  }
}

// Buffer descriptor of one FP32 plane of `bytes` bytes (raw: stride 0,
// GFX9 dword-3 format word), and a dword load at vector offset `vo` plus
// scalar offset `so`.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, bytes, 0x00020000);
}
__device__ __forceinline__ float plane_load(__amdgpu_buffer_rsrc_t rs, int vo, int so) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, vo, so, 0));
}

// Rows y0 .. y0 + NV - 1 of one column of an FP32 plane (byte offset xb of
// the column; zero outside the image or where !xin).
template <int NV>
__device__ __forceinline__ void column_block(const float* plane, int bytes, int xb, int y0, int H,
                                             int W, bool xin, float (&v)[NV]) {
  const __amdgpu_buffer_rsrc_t rs = plane_rsrc(plane, bytes);
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int y = y0 + i;
    const float t = plane_load(rs, xb, min(max(y, 0), H - 1) * W * 4);
    const unsigned keep = (xin && y >= 0 && y < H) ? 0xffffffffu : 0u;
    v[i] = __uint_as_float(__float_as_uint(t) & keep);
  }
}

// Raw FP32 guides and noisy values of one pixel (zeros outside the image),
// and their conversion to the shifted sum type. Split so that the loads for
// the next row can be issued a whole iteration before they are consumed.
template <int Q, int C>
__device__ __forceinline__ void load_raw(const LaunchArgs& a, int64_t pl, int64_t off, bool ok,
                                         float (&v)[Q + C]) {
  if (ok) {
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = a.guides[q * pl + off];
#pragma unroll
    for (int c = 0; c < C; ++c) v[Q + c] = a.noisy[c * pl + off];
  } else {
#pragma unroll
    for (int i = 0; i < Q + C; ++i) v[i] = 0.f;
  }
}
template <int Q, int C>
__device__ __forceinline__ void shift_raw(const float (&v)[Q + C], bool ok, const float (&cg)[Q],
                                          sum_t (&g)[Q], sum_t (&y)[C]) {
#pragma unroll
  for (int q = 0; q < Q; ++q) g[q] = ok ? (sum_t)v[q] - (sum_t)cg[q] : sum_t(0);
#pragma unroll
  for (int c = 0; c < C; ++c) y[c] = (sum_t)v[Q + c];
}

// Channel order: sum g[Q] | sum y[C] | sum g_p g_q (p<=q) | sum g_q y_c.
// A walker may carry only a slice of the product channels: products
// [POFF, POFF + PCNT) of the Q(Q+1)/2 + QC, after the Q + C first moments,
// which every walker carries. chan_local maps a channel to its index in
// the walker (-1 when outside the slice); it folds at compile time.
template <int Q, int C, int POFF, int PCNT>
__host__ __device__ constexpr int chan_local(int m) {
  return m < Q + C ? m : ((m - Q - C >= POFF && m - Q - C < POFF + PCNT) ? m - POFF : -1);
}

// V += products of the entering pixel (ga, ya) - those of the leaving one.
template <int Q, int C, int POFF, int PCNT>
__device__ __forceinline__ void vupdate(sum_t (&V)[Q + C + PCNT], const sum_t (&ga)[Q],
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
      const int l = chan_local<Q, C, POFF, PCNT>(k);
      if (l >= 0) V[l] = fma_t(-gs[p], gs[q], fma_t(ga[p], ga[q], V[l]));
      ++k;
    }
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int l = chan_local<Q, C, POFF, PCNT>(k);
      if (l >= 0) V[l] = fma_t(-gs[q], ys[c], fma_t(ga[q], ya[c], V[l]));
      ++k;
    }
  }
}

// Change of channels [g0, g0 + gn) of the running vertical sums when the
// entering pixel (ga, ya) is added and the leaving one (gs, ys) removed
// (channel order as in vupdate); every index folds at compile time.
template <int Q, int C, int MG, int POFF, int PCNT>
__device__ __forceinline__ void group_deltas(int g0, int gn, const sum_t (&ga)[Q],
                                             const sum_t (&ya)[C], const sum_t (&gs)[Q],
                                             const sum_t (&ys)[C], sum_t (&dl)[MG]) {
  // local index of channel m within [g0, g0 + gn), else -1
  auto at = [&](int m) {
    const int l = chan_local<Q, C, POFF, PCNT>(m);
    return (l >= g0 && l < g0 + gn) ? l - g0 : -1;
  };
#pragma unroll
  for (int q = 0; q < Q; ++q)
    if (at(q) >= 0) dl[at(q)] = ga[q] - gs[q];
#pragma unroll
  for (int c = 0; c < C; ++c)
    if (at(Q + c) >= 0) dl[at(Q + c)] = ya[c] - ys[c];
  int k = Q + C;
#pragma unroll
  for (int p = 0; p < Q; ++p) {
#pragma unroll
    for (int q = p; q < Q; ++q) {
      if (at(k) >= 0) dl[at(k)] = fma_t(-gs[p], gs[q], ga[p] * ga[q]);
      ++k;
    }
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (at(k) >= 0) dl[at(k)] = fma_t(-gs[q], ys[c], ga[q] * ya[c]);
      ++k;
    }
  }
}

// LDS byte addresses of the three prefix terms of a window (HWin) in a
// group of prefix rows starting at P: for channels 0..31 of the group and,
// through a second base with the same immediates, for channels 32 and up, so
// that every read is a base register plus an immediate offset below 64 KB.
// The bases pass through lane_opaque so that they are formed once per row
// rather than hoisted out of the row loop as one address per channel. Every
// lane of the wavefront must call it (DPP).
constexpr int kGroupBase = 32;  // channels per base
struct GroupAddr {
  int b[2], a[2], t[2];
};
__device__ __forceinline__ GroupAddr group_addr(const sum_t* P, const HWin& h) {
  extern __shared__ float lds[];
  const int o0 = (int)(reinterpret_cast<const char*>(P) - reinterpret_cast<const char*>(lds));
  constexpr int RB = kLdsStride * (int)sizeof(sum_t);  // bytes per prefix row
  constexpr int E = (int)sizeof(sum_t);
  GroupAddr g;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int o = o0 + j * kGroupBase * RB;
    g.b[j] = lane_opaque(o + h.ib * E);
    g.a[j] = lane_opaque(o + h.ia * E);
    g.t[j] = lane_opaque(o + h.it * E);
  }
  return g;
}
__device__ __forceinline__ sum_t group_read(const int (&base)[2], int m) {
  extern __shared__ float lds[];
  constexpr int RB = kLdsStride * (int)sizeof(sum_t);
  return *reinterpret_cast<const sum_t*>(reinterpret_cast<const char*>(lds) +
                                         base[m / kGroupBase] + (m % kGroupBase) * RB);
}

// Fold the window sums of channels [g0, g0 + gn) (one LDS group of segment
// prefixes, row stride kLdsStride, read through the addresses `ga`) into the
// central moments: mu~, nu, the guide covariance Hm and the guide/channel
// covariance R. Channel order: sum g | sum y | sum g_p g_q (p <= q) |
// sum g_q y_c (shifted guides). Groups arrive in increasing order and the
// first holds all Q + C first moments, so the means are complete before any
// covariance needs them. All loops unroll and every group test folds at
// compile time.
template <int Q, int C, int MG, int POFF, int PCNT, typename T, typename U>
__device__ __forceinline__ void centre_group(int g0, int gn, const GroupAddr& ga, T inv_n,
                                             T (&mu)[Q], T (&nu)[C],
                                             U (&Hm)[Q * (Q + 1) / 2], U (&R)[Q * C]) {
  constexpr int NP = Q * (Q + 1) / 2;
  // window sums of the group: the three prefix reads of four channels are
  // issued together, ahead of their arithmetic
  constexpr int B = 4;
  T ws[MG];
#pragma unroll
  for (int k0 = 0; k0 < MG; k0 += B) {
    sum_t rb[B], ra[B], rt[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
      if (k0 + i < gn) {
        rb[i] = group_read(ga.b, k0 + i);
        ra[i] = group_read(ga.a, k0 + i);
        rt[i] = group_read(ga.t, k0 + i);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < B; ++i)
      if (k0 + i < gn) ws[k0 + i] = (T)((rb[i] - ra[i]) + rt[i]);
  }
  // index into ws of channel m when it is in this group, else -1
  auto at = [&](int m) {
    const int l = chan_local<Q, C, POFF, PCNT>(m);
    return (l >= g0 && l < g0 + gn) ? l - g0 : -1;
  };
#pragma unroll
  for (int q = 0; q < Q; ++q)
    if (at(q) >= 0) mu[q] = ws[at(q)] * inv_n;
#pragma unroll
  for (int c = 0; c < C; ++c)
    if (at(Q + c) >= 0) nu[c] = ws[at(Q + c)] * inv_n;
#pragma unroll
  for (int p = 0; p < Q; ++p) {
#pragma unroll
    for (int q = p; q < Q; ++q) {
      const int m = Q + C + tri<Q>(p, q);
      if (at(m) >= 0) Hm[tri<Q>(p, q)] = (U)fma_t(ws[at(m)], inv_n, -mu[p] * mu[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int m = Q + C + NP + q * C + c;
      if (at(m) >= 0) R[q * C + c] = (U)fma_t(ws[at(m)], inv_n, -mu[q] * nu[c]);
    }
  }
}

// Horizontal sums of the F*C coefficient rows held in LDS (t0, written by
// the caller in groups via `fill`), and the reconstruction
//   out_c = (sum b~_c + sum_q g~_q sum a_qc) / n   for output lane `o`.
// `fill(f0, gn, t0)` writes coefficient rows f0..f0+gn-1 into t0.
template <int Q, int C, int AG, typename Fill>
__device__ __forceinline__ void average_and_reconstruct(solve_t* t0, solve_t* t1, int nout, int r,
                                                        int chunk, bool active,
                                                        const solve_t (&gq)[Q], solve_t inv_n,
                                                        float* out_c0, int64_t pl, Fill fill) {
  constexpr int FC = Dims<Q, C>::FC;
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

// Reconstruction from the window sums of all F*C coefficient rows (column
// base `col`): out_c = (sum b~_c + sum_q g~_q sum a_qc) / n.
template <int Q, int C>
__device__ __forceinline__ void reconstruct(const solve_t* col, bool active, const solve_t (&gq)[Q],
                                            solve_t inv_n, float* out_c0, int64_t pl) {
  if (!active) return;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    solve_t acc = col[c * kLdsStride];
#pragma unroll
    for (int q = 0; q < Q; ++q) acc = fma_t(gq[q], col[((1 + q) * C + c) * kLdsStride], acc);
    out_c0[c * pl] = (float)(acc * inv_n);
  }
}

enum WalkMode : int { W_MOMENTS = 0, W_FUSED0 = 1, W_FUSED1 = 2, W_COEFFS = 3, W_SPLITSOLVE = 4 };

// ---------------------------------------------------------------------------
// The walker. MODE selects what happens with the window moments of each
// coefficient position:
//   W_MOMENTS  write the moment planes (central, or raw sums with a.raw);
//   W_FUSED0   solve and reconstruct at the same pixel;
//   W_COEFFS   solve and write the coefficient planes (original units);
//   W_SPLITSOLVE  (split walks, the second slice) read the first slice's
//              central moments from the moment planes of the walk over it
//              (a.planes), then as W_COEFFS;
//   W_FUSED1   solve, push the coefficients through a per-workgroup ring of
//              2r+1 rows (global workspace) to form vertical window sums,
//              stage those through LDS for the horizontal sums, and
//              reconstruct with the averaged coefficients. The segment is
//              extended by r coefficient rows above and below and the strip
//              by r columns each side, so no data crosses workgroups.
// POFF, PCNT: the slice of product channels this walker carries (all by
// default); W_MOMENTS over a slice writes that slice's planes (and, for the
// first slice, n and the means).
// The frame and local workgroup index of a batched launch (frames are few:
// a scan of the workgroup offsets, uniform across the workgroup).
__device__ __forceinline__ const LaunchArgs& batch_frame(const LaunchArgs& ain, int* bid) {
  const int b = blockIdx.x;
  int f = 0;
  while (f + 1 < ain.nframes && ain.wg_start[f + 1] <= b) ++f;
  *bid = b - ain.wg_start[f];
  return ain.frames[f];
}

// One workgroup's tile (strip sx = bid % tiles_x, segment bid / tiles_x) of
// frame a.
template <int Q, int C, int MODE, bool WIDE, int POFF = 0, int PCNT = -1>
__device__ __forceinline__ void walk_tile(const LaunchArgs a, const int bid) {
  using D = Dims<Q, C>;
  using T = solve_t;
  constexpr int NPQ = D::NP + D::NQC;              // product channels
  constexpr int PC = PCNT < 0 ? NPQ : PCNT;
  constexpr int NS = Q + C + PC;                   // channels of this walker
  constexpr int FC = D::FC;
  constexpr int NP = D::NP;
  constexpr WalkLayout LAY = walk_layout(
      Q, C,
      MODE == W_FUSED1 ? K_FUSED1
                       : (MODE == W_FUSED0 ? K_FUSED0 : (MODE == W_MOMENTS ? K_MOMENTS : K_COEFFS)),
      NS);
  constexpr int MG = LAY.mg;
  constexpr bool VA_LDS = MODE == W_FUSED1 && LAY.va_lds;
  extern __shared__ float lds[];
  char* lb = reinterpret_cast<char*>(lds);
  sum_t* S0 = reinterpret_cast<sum_t*>(lb);
  sum_t* S1 = reinterpret_cast<sum_t*>(lb + LAY.a);
  T* T0 = reinterpret_cast<T*>(lb);
  T* T1 = reinterpret_cast<T*>(lb + LAY.a);
  T* VAL = reinterpret_cast<T*>(lb + LAY.a + LAY.b);  // VA_LDS: [FC][kLdsStride]

  const int tid = threadIdx.x;
  const int r = a.r;
  const int H = a.H;
  const int W = a.W;
  const int64_t pl = (int64_t)H * W;
  const int hc = MODE == W_FUSED1 ? r : 0;
  const int ncoef = kThreads - 2 * r;
  const int tout = ncoef - 2 * hc;
  const int sx = bid % a.tiles_x;
  const int sy = bid / a.tiles_x;
  const int X0 = sx * tout;
  const int Y0 = sy * a.seg_rows;
  const int Y1 = min(Y0 + a.seg_rows, H);
  const int xi = X0 - hc - r + tid;  // input column of this lane
  const bool xin = xi >= 0 && xi < W;
  const int xc = X0 - hc + tid;      // coefficient column of this lane (tid < ncoef)
  const bool cvalid = tid < ncoef && xc >= 0 && xc < W;
  constexpr int NG = (NS + MG - 1) / MG;  // LDS groups of moment channels
  // With at most two groups, every channel's segment prefix stays resident
  // in LDS from one row to the next, and the running vertical sums are
  // recovered from it (V[j] = P[j] - P[j-1] within a segment) instead of
  // being held in registers across the row.
  constexpr bool VL = MODE != W_FUSED1 && NG <= 2;
  constexpr int IL = 4;  // channels whose lane moves interleave
  const HWin hw = hwin<WIDE>(tid, r);
  // zero pad column of every prefix row of both buffers (no other pass
  // writes column kThreads; the first group's barrier orders these stores)
  for (int m = tid; m < 2 * MG; m += kThreads) (m < MG ? S0 : S1)[(m % MG) * kLdsStride + kThreads] = sum_t(0);

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
    // warm-up: rows [ym0 - r, ym0 + r) of the first window, each row's loads
    // issued one step ahead
    sum_t zg[Q], zy[C];
#pragma unroll
    for (int q = 0; q < Q; ++q) zg[q] = sum_t(0);
#pragma unroll
    for (int c = 0; c < C; ++c) zy[c] = sum_t(0);
    float wb[Q + C];
    bool wok = xin && ym0 - r >= 0 && ym0 - r < H;
    load_raw<Q, C>(a, pl, (int64_t)(ym0 - r) * W + xi, wok, wb);
    for (int yy = ym0 - r; yy < ym0 + r; ++yy) {
      float cur[Q + C];
#pragma unroll
      for (int i = 0; i < Q + C; ++i) cur[i] = wb[i];
      const bool cok = wok;
      if (yy + 1 < ym0 + r) {
        wok = xin && yy + 1 >= 0 && yy + 1 < H;
        load_raw<Q, C>(a, pl, (int64_t)(yy + 1) * W + xi, wok, wb);
      }
      sum_t g[Q], y[C];
      shift_raw<Q, C>(cur, cok, cg, g, y);
      vupdate<Q, C, POFF, PC>(V, g, y, zg, zy);
    }
  }

  if (VL) {
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
      const int g0 = gi * MG;
      const int gn = NS - g0 < MG ? NS - g0 : MG;
      sum_t* P = (gi & 1) ? S1 : S0;
#pragma unroll
      for (int m0 = 0; m0 < gn; m0 += IL) {
        sum_t x[IL];
#pragma unroll
        for (int i = 0; i < IL; ++i) x[i] = m0 + i < gn ? V[g0 + m0 + i] : sum_t(0);
        seg_prefix_n<WIDE>(x);
#pragma unroll
        for (int i = 0; i < IL; ++i)
          if (m0 + i < gn) P[(m0 + i) * kLdsStride + tid] = x[i];
      }
    }
  }

  constexpr int NVA = (MODE == W_FUSED1 && !VA_LDS) ? FC : 1;
  avg_t Va[NVA];
#pragma unroll
  for (int f = 0; f < NVA; ++f) Va[f] = avg_t(0);
  if (VA_LDS) {
#pragma unroll
    for (int f = 0; f < FC; ++f) VAL[f * kLdsStride + tid] = T(0);
  }
  // the workgroup's ring (K_FUSED1 only; no ring otherwise)
  ring_t* ring = a.ring ? reinterpret_cast<ring_t*>(a.ring) +
                              (size_t)bid * (size_t)(2 * r + 1) * FC * kThreads + tid
                        : nullptr;

  // inputs of the rows entering (ym + r) and leaving (ym - r - 1) the window
  float fa[Q + C], fs[Q + C];
  bool okA = false, okS = false;
  auto fetch = [&](int y) {
    const int ya = y + r;
    const int ys = y - r - 1;
    okA = xin && ya >= 0 && ya < H;
    okS = xin && y > ym0 && ys >= 0 && ys < H;
    load_raw<Q, C>(a, pl, (int64_t)ya * W + xi, okA, fa);
    load_raw<Q, C>(a, pl, (int64_t)ys * W + xi, okS, fs);
  };
  fetch(ym0);

  // Coefficient ring (K_FUSED1, r > 0): oldv holds the values of the row
  // leaving the vertical average at the current step. The reads for the next
  // step are issued after this step's use but before this step's ring
  // stores, so that waiting for them never waits on recent stores (vector
  // memory operations retire in issue order).
  constexpr int NRING = MODE == W_FUSED1 ? FC : 1;
  ring_t oldv[NRING];
  auto ring_fetch = [&](int y) {
    const int yold = y - 2 * r - 1;
    const bool ok = MODE == W_FUSED1 && r > 0 && tid < ncoef && y < ym1 && yold >= ym0 &&
                    yold >= 0 && yold < H;
    const ring_t* rs = ring + (size_t)((y - ym0) % (2 * r + 1)) * FC * kThreads;
#pragma unroll
    for (int f = 0; f < NRING; ++f) oldv[f] = ok ? rs[f * kThreads] : ring_t(0);
  };
  ring_fetch(ym0);

  for (int ym = ym0; ym < ym1; ++ym) {
    sum_t ga[Q], yA[C], gs[Q], yS[C];
    shift_raw<Q, C>(fa, okA, cg, ga, yA);
    shift_raw<Q, C>(fs, okS, cg, gs, yS);
    if (!VL) vupdate<Q, C, POFF, PC>(V, ga, yA, gs, yS);
    if (ym + 1 < ym1) fetch(ym + 1);

    const int slot = MODE == W_FUSED1 ? (ym - ym0) % (2 * r + 1) : 0;
    const bool row_in = ym >= 0 && ym < H;

    constexpr int NCV = MODE == W_FUSED1 ? FC : 1;
    T cv[NCV];
#pragma unroll
    for (int f = 0; f < NCV; ++f) cv[f] = T(0);

    if (row_in) {
      const int64_t off = (int64_t)ym * W + xc;
      const int ni = cvalid ? win_count(ym, H, r) * win_count(xc, W, r) : 1;
      const T inv_n = recip_count(ni, T(0));
      // means in solve_t; the centred system (formed in solve_t) in chol_t
      T mu[Q], nu[C];
      chol_t Hm[NP], R[Q * C];

      // Groups of channels alternate between the two LDS buffers, so one
      // barrier per group separates its prefix writes from its window reads
      // and the reads of the group before last from this group's writes.
      // With an odd group count the first buffer of a row is the one the
      // previous row's last group read, hence the extra barrier. (Writing
      // both groups before reading either was measured in the assembly: the
      // compiler then keeps more values live and spills more.)
      if (NG % 2 == 1) __syncthreads();
      const HWin hr = hwin_opaque(hw);  // this row's window addresses
      // prefixes of group gi's channels into its buffer
      auto walk_group = [&](const int gi) {
        const int g0 = gi * MG;
        const int gn = NS - g0 < MG ? NS - g0 : MG;
        sum_t* P = (gi & 1) ? S1 : S0;
        // VL: the previous row's prefixes of each chunk, read one chunk ahead
        sum_t nx[IL];
        if (VL) {
#pragma unroll
          for (int i = 0; i < IL; ++i) nx[i] = i < gn ? P[i * kLdsStride + tid] : sum_t(0);
        }
#pragma unroll
        for (int m0 = 0; m0 < gn; m0 += IL) {
          sum_t x[IL];
          if (VL) {
            // The segment prefix of the vertical sums telescopes: this row's
            // prefix is the previous row's (own column, read one chunk
            // ahead) plus the segment prefix of this row's change.
#pragma unroll
            for (int i = 0; i < IL; ++i) x[i] = nx[i];
#pragma unroll
            for (int i = 0; i < IL; ++i)
              nx[i] = m0 + IL + i < gn ? P[(m0 + IL + i) * kLdsStride + tid] : sum_t(0);
            __builtin_amdgcn_sched_barrier(0);
            sum_t dl[IL];  // this row's change of the chunk's channels
            group_deltas<Q, C, IL, POFF, PC>(g0 + m0, gn - m0 < IL ? gn - m0 : IL, ga, yA, gs, yS, dl);
#pragma unroll
            for (int i = 0; i < IL; ++i) dl[i] = m0 + i < gn ? dl[i] : sum_t(0);
            seg_prefix_n<WIDE>(dl);
#pragma unroll
            for (int i = 0; i < IL; ++i) x[i] += dl[i];
          } else {
#pragma unroll
            for (int i = 0; i < IL; ++i) x[i] = m0 + i < gn ? V[g0 + m0 + i] : sum_t(0);
            seg_prefix_n<WIDE>(x);
          }
#pragma unroll
          for (int i = 0; i < IL; ++i)
            if (m0 + i < gn) P[(m0 + i) * kLdsStride + tid] = x[i];
        }
      };
      // window sums of group gi's channels: written out, or centred
      auto read_group = [&](const int gi) {
        const int g0 = gi * MG;
        const int gn = NS - g0 < MG ? NS - g0 : MG;
        const sum_t* P = (gi & 1) ? S1 : S0;
        const GroupAddr gad = group_addr(P, hw);  // every lane (DPP)
        if (cvalid) {
          if (MODE == W_MOMENTS && a.raw) {
#pragma unroll
            for (int m = 0; m < gn; ++m) {
              const int l = g0 + m;  // local channel -> global channel
              const int gch = l < Q + C ? l : l + POFF;
              if (POFF == 0 || l >= Q + C)
                a.out[(1 + gch) * pl + off] = (float)hwin_sum(P + m * kLdsStride, hr);
            }
          } else {
            centre_group<Q, C, MG, POFF, PC, T, chol_t>(g0, gn, gad, inv_n, mu, nu, Hm, R);
          }
        }
      };
#pragma unroll
      for (int gi = 0; gi < NG; ++gi) {
        walk_group(gi);
        __syncthreads();
        read_group(gi);
      }
      if (cvalid) {
        if (MODE == W_MOMENTS) {
          // a slice writes its own product planes; the first one also n, mu, nu
          if (POFF == 0) a.out[off] = (float)ni;
          if (!a.raw) {
            if (POFF == 0) {
#pragma unroll
              for (int q = 0; q < Q; ++q) a.out[(1 + q) * pl + off] = (float)(mu[q] + (T)cg[q]);
#pragma unroll
              for (int c = 0; c < C; ++c) a.out[(1 + Q + c) * pl + off] = (float)nu[c];
            }
#pragma unroll
            for (int k = POFF; k < POFF + PC; ++k)
              a.out[(1 + Q + C + k) * pl + off] = k < NP ? (float)Hm[k] : (float)R[k - NP];
          }
        } else {
          if constexpr (MODE == W_SPLITSOLVE) {
            // the first slice's product channels: central moments written by
            // the walk over that slice (shift-free, so the anchors agree)
#pragma unroll
            for (int k = 0; k < POFF; ++k) {
              const chol_t v = (chol_t)a.planes[(int64_t)(1 + Q + C + k) * pl + off];
              if (k < NP)
                Hm[k] = v;
              else
                R[k - NP] = v;
            }
          }
          T mu_o[Q];
          chol_t mu_c[Q];
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            mu_o[q] = mu[q] + (T)cg[q];
            mu_c[q] = (chol_t)mu_o[q];
          }
          regularise<Q, chol_t>(Hm, mu_c, (chol_t)arg_eps(a), (chol_t)arg_eps_mul(a), a.reg_mode);
          chol_solve<Q, C, chol_t>(Hm, R);
          if (MODE == W_COEFFS || MODE == W_SPLITSOLVE) {
            // b = nu - a^T mu in original units
            if (a.coef_lo) {
              // from the slopes as stored, kept as hi + lo
#pragma unroll
              for (int c = 0; c < C; ++c) {
                T b = nu[c];
#pragma unroll
                for (int q = 0; q < Q; ++q) b = fma_t(-(T)(float)R[q * C + c], mu_o[q], b);
                const float hi = (float)b;
                a.out[c * pl + off] = hi;
                a.out[((Q + 1) * C + c) * pl + off] = (float)(b - (T)hi);
              }
            } else {
#pragma unroll
              for (int c = 0; c < C; ++c) {
                T b = nu[c];
#pragma unroll
                for (int q = 0; q < Q; ++q) b = fma_t(-(T)R[q * C + c], mu_o[q], b);
                a.out[c * pl + off] = (float)b;
              }
            }
#pragma unroll
            for (int k = 0; k < Q * C; ++k) a.out[(C + k) * pl + off] = (float)R[k];
          } else if (MODE == W_FUSED0) {
            T gp[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) gp[q] = ((T)a.guides[q * pl + off] - (T)cg[q]) - mu[q];
#pragma unroll
            for (int c = 0; c < C; ++c) {
              T acc = nu[c];
#pragma unroll
              for (int q = 0; q < Q; ++q) acc = fma_t(gp[q], (T)R[q * C + c], acc);
              a.out[c * pl + off] = (float)acc;
            }
          } else {
            // coefficients relative to the anchor: b~ = nu - a^T mu~
#pragma unroll
            for (int c = 0; c < C; ++c) {
              T b = nu[c];
#pragma unroll
              for (int q = 0; q < Q; ++q) b = fma_t(-(T)R[q * C + c], mu[q], b);
              cv[c] = b;
            }
#pragma unroll
            for (int k = 0; k < Q * C; ++k) cv[C + k] = (T)R[k];
          }
        }
      }
    }

    if (MODE == W_FUSED1) {
      // vertical window sums of the coefficients through the ring
      if (tid < ncoef) {
#pragma unroll
        for (int f = 0; f < FC; ++f) {
          // the ring holds the stored (rounded) values, so add those too
          const ring_t nw = (ring_t)cv[f];
          if (r == 0) {  // window of one row: no history needed
            if (VA_LDS)
              VAL[f * kLdsStride + tid] = (T)nw;
            else
              Va[f] = (avg_t)nw;
          } else if (VA_LDS) {
            VAL[f * kLdsStride + tid] += (T)nw - (T)oldv[f];
          } else {
            Va[f] += (avg_t)nw - (avg_t)oldv[f];
          }
        }
      }
      ring_fetch(ym + 1);
      if (tid < ncoef && row_in && r > 0) {
        ring_t* rs = ring + (size_t)slot * FC * kThreads;
#pragma unroll
        for (int f = 0; f < FC; ++f) rs[f * kThreads] = (ring_t)cv[f];
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
          inv = recip_count(win_count(yo, H, r) * win_count(xo, W, r), T(0));
        } else {
#pragma unroll
          for (int q = 0; q < Q; ++q) gq[q] = T(0);
        }
        if (VA_LDS) {
          __syncthreads();
          hbox(VAL, T1, FC, tout, r, a.hchunk_a);
          __syncthreads();
          reconstruct<Q, C>(T1 + tid, active, gq, inv, a.out + off, pl);
        } else {
          average_and_reconstruct<Q, C, LAY.ag>(
              T0, T1, tout, r, a.hchunk_a, active, gq, inv, a.out + off, pl,
              [&](int f0, int gn, T* dst) {
                if (tid < ncoef) {
#pragma unroll
                  for (int k = 0; k < gn; ++k) dst[k * kLdsStride + tid] = (T)Va[f0 + k];
                }
              });
        }
      }
    }
  }
}

template <int Q, int C, int MODE, bool WIDE, int POFF = 0, int PCNT = -1, bool BATCH = false>
__global__ void __launch_bounds__(kThreads, 1) walk_kernel(LaunchArgs ain) {
  int bid = blockIdx.x;
  const LaunchArgs a = BATCH ? batch_frame(ain, &bid) : ain;
  walk_tile<Q, C, MODE, WIDE, POFF, PCNT>(a, bid);
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
  regularise<Q, T>(Hm, mu, (T)arg_eps(a), (T)arg_eps_mul(a), a.reg_mode);
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
    if (a.coef_lo) acc += (T)a.planes[((Q + 1) * C + c) * pl + idx];
#pragma unroll
    for (int q = 0; q < Q; ++q) acc = fma_t(g[q], (T)a.planes[((1 + q) * C + c) * pl + idx], acc);
    a.out[c * pl + idx] = (float)acc;
  }
}

// flr_apply with averaging (Sec. 3.1: each pixel's output uses the mean of
// the coefficients of the windows that contain it). A workgroup owns a tile
// of th <= kAvgTileRows output rows by 256 - 2r output columns; lane l owns
// input column X0 - r + l. The coefficient planes are taken one at a time:
// the lane streams its column's th + 2r rows of the plane once, forms the
// vertical window sums of the tile's rows by sliding (FP64), and the
// horizontal sums come from DPP segment prefixes staged in LDS, as in the
// moment walkers. Each output lane accumulates
//   out_c = (sum b_c + sum_q g_q * sum a_qc) / n
// for all C channels of its th pixels in FP64 registers. Planes alternate
// between two LDS buffers, one barrier each.
// Variants of the averaging kernel: the column walk streams its rows for any
// radius (AV_STREAM16: 16-lane prefix segments, r <= 8; AV_STREAM64:
// wavefront segments, r > 8), or, for r = 8 and up to three channels (the
// register budget of two workgroups per CU), loads each plane's column
// block once and slides with compile-time offsets (AV_BLOCK8).
enum AvgVariant : int { AV_STREAM16 = 0, AV_STREAM64 = 1, AV_BLOCK8 = 2 };
__host__ __device__ constexpr int avg_variant(int r, int C) {
  return (r == 8 && C <= 3) ? AV_BLOCK8 : (wide_segments(r) ? AV_STREAM64 : AV_STREAM16);
}

template <int Q, int C, int AV, bool LO>
__device__ __forceinline__ void apply_avg_tile(const LaunchArgs a, const int sx, const int sy) {
  using T = solve_t;
  constexpr bool WIDE = AV == AV_STREAM64;
  constexpr int TH = kAvgTileRows;
  extern __shared__ float lds[];
  T* P0 = reinterpret_cast<T*>(lds);
  T* P1 = P0 + TH * kLdsStride;
  const int tid = threadIdx.x;
  const int r = a.r;
  const int H = a.H;
  const int W = a.W;
  const int64_t pl = (int64_t)H * W;
  const int tout = kThreads - 2 * r;
  const int X0 = sx * tout;
  const int Y0 = sy * a.seg_rows;
  const int th = min(a.seg_rows, H - Y0);
  const int xcol = X0 - r + tid;
  const bool xin = xcol >= 0 && xcol < W;
  const int xo = X0 + tid;
  const bool active = tid < tout && xo < W;
  const HWin hw = hwin<WIDE>(tid, r);
  if (tid < 2 * TH) (tid < TH ? P0 : P1)[(tid % TH) * kLdsStride + kThreads] = T(0);

  T acc[TH][C];
#pragma unroll
  for (int k = 0; k < TH; ++k)
#pragma unroll
    for (int c = 0; c < C; ++c) acc[k][c] = T(0);

  // Loads use clamped, always valid addresses (a plane base pointer plus a
  // 32-bit offset) and zero what lies outside the image by selection, so
  // that no load needs a branch.
  // Raw buffer loads: a descriptor per plane, the lane's column byte offset
  // (vector) and the row's byte offset (scalar; rows are clamped into the
  // image, so every access is in range; planes hold at most 2^28 pixels, so
  // offsets fit in 32 bits).
  const int xcb = min(max(xcol, 0), W - 1) * 4;
  const int xob = min(xo, W - 1) * 4;
  const int pbytes = (int)(pl * 4 <= 0x7fffffff ? pl * 4 : 0x7fffffff);
  auto at = [&](const float* base, int y, int xb) {
    const int so = min(max(y, 0), H - 1) * W * 4;
    return plane_load(plane_rsrc(base, pbytes), xb, so);
  };
  // Window sums of the tile's rows from the prefixes in P, batched four
  // rows (twelve reads) at a time, accumulated into channel c's sums.
  auto consume = [&](const T* P, int c, bool plain, const float (&gf)[TH]) {
    constexpr int B = 4;
#pragma unroll
    for (int k0 = 0; k0 < TH; k0 += B) {
      T rb[B], ra[B], rt[B];
#pragma unroll
      for (int i = 0; i < B; ++i) {
        if (k0 + i < TH) {
          const T* row = P + (k0 + i) * kLdsStride;
          rb[i] = row[hw.ib];
          ra[i] = row[hw.ia];
          rt[i] = row[hw.it];
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < B; ++i) {
        if (k0 + i < TH) {
          const T v = (rb[i] - ra[i]) + rt[i];
#pragma unroll
          for (int cc = 0; cc < C; ++cc)
            if (cc == c)
              acc[k0 + i][cc] = plain ? acc[k0 + i][cc] + v : fma_t((T)gf[k0 + i], v, acc[k0 + i][cc]);
        }
      }
    }
  };
  // DPP segment prefixes of the tile's vertical sums into LDS buffer P
  auto stage = [&](T* P, const T (&vs)[TH]) {
    constexpr int IL = 4;
#pragma unroll
    for (int k0 = 0; k0 < TH; k0 += IL) {
      T x[IL];
#pragma unroll
      for (int i = 0; i < IL; ++i) x[i] = k0 + i < TH ? vs[k0 + i] : T(0);
      seg_prefix_n<WIDE>(x);
#pragma unroll
      for (int i = 0; i < IL; ++i)
        if (k0 + i < TH) P[(k0 + i) * kLdsStride + tid] = x[i];
    }
  };
  auto load_gf = [&](int q, float (&gf)[TH]) {
    const float* g = a.guides + (int64_t)q * pl;
#pragma unroll
    for (int k = 0; k < TH; ++k) gf[k] = at(g, Y0 + k, xob);
  };

  // planes: b (C), a (Q C), then with LO the intercepts' lo parts (C),
  // taken as a pass q = Q that adds like the intercepts
  constexpr int qend = LO ? Q + 1 : Q;
  constexpr int nplanes = (qend + 1) * C;
  int buf = 0;
  if constexpr (AV == AV_BLOCK8) {
    // r = 8: the lane loads its column's rows Y0 - 8 .. Y0 + TH + 7 of a
    // plane as one block (zero outside the image), issued while the plane
    // before it is staged and consumed.
    constexpr int NV = TH + 16;
    auto load_block = [&](int f, float (&v)[NV]) {
      column_block<NV>(a.planes + (int64_t)f * pl, pbytes, xcb, Y0 - 8, H, W, xin, v);
    };
    // vertical window sums of rows Y0 + k: rows Y0 + k - R .. Y0 + k + R
    auto slide = [&](auto RC, const float (&v)[NV], T (&vs)[TH]) {
      constexpr int R = decltype(RC)::value;
      T sum = T(0);
#pragma unroll
      for (int i = 8 - R; i <= 8 + R; ++i) sum += (T)v[i];
      vs[0] = sum;
#pragma unroll
      for (int k = 1; k < TH; ++k) {
        sum += (T)v[k + 8 + R] - (T)v[k + 7 - R];
        vs[k] = sum;
      }
    };
    float cur[NV];
    load_block(0, cur);
    float gf[TH];
    for (int q = -1; q < qend; ++q) {
      if (q >= 0 && q < Q) load_gf(q, gf);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int f = (q + 1) * C + c;
        T vs[TH];
        slide(std::integral_constant<int, 8>{}, cur, vs);
        // the next plane's block streams in during staging and consumption
        if (f + 1 < nplanes) load_block(f + 1, cur);
        T* P = buf ? P1 : P0;
        buf ^= 1;
        stage(P, vs);
        __syncthreads();
        if (active) consume(P, c, q < 0 || q == Q, gf);
      }
    }
  } else {
    // any r: the window of the tile's first row is summed by a running
    // loop; rows entering and leaving are loaded for each later row.
    float gf[TH];
    for (int q = -1; q < qend; ++q) {
      if (q >= 0 && q < Q) load_gf(q, gf);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const float* src = a.planes + (int64_t)((q + 1) * C + c) * pl;
        T sum = T(0);
        for (int y = max(Y0 - r, 0); y <= min(Y0 + r, H - 1); ++y) sum += (T)at(src, y, xcb);
        if (!xin) sum = T(0);
        T vs[TH];
        vs[0] = sum;
#pragma unroll
        for (int k = 1; k < TH; ++k) {
          const int ye = Y0 + r + k, yl = Y0 - r - 1 + k;
          const float ve = at(src, ye, xcb), vl = at(src, yl, xcb);
          const float e = (xin && k < th && ye < H) ? ve : 0.f;
          const float l = (xin && k < th && yl >= 0) ? vl : 0.f;
          sum += (T)e - (T)l;
          vs[k] = sum;
        }
        T* P = buf ? P1 : P0;
        buf ^= 1;
        stage(P, vs);
        __syncthreads();
        if (active) consume(P, c, q < 0 || q == Q, gf);
      }
    }
  }
  if (active) {
#pragma unroll
    for (int k = 0; k < TH; ++k) {
      if (k < th) {
        const int y = Y0 + k;
        const T inv = recip_count(win_count(y, H, r) * win_count(xo, W, r), T(0));
        float* o = a.out + (int64_t)y * W + xo;
#pragma unroll
        for (int c = 0; c < C; ++c) o[c * pl] = (float)(acc[k][c] * inv);
      }
    }
  }
}

template <int Q, int C, int AV>
__device__ __forceinline__ void apply_avg_tile_any(const LaunchArgs& a, const int sx,
                                                   const int sy) {
  if (a.coef_lo)
    apply_avg_tile<Q, C, AV, true>(a, sx, sy);
  else
    apply_avg_tile<Q, C, AV, false>(a, sx, sy);
}

// Tile of averaging workgroup b of a frame's launch range. Workgroups are
// dealt to the XCDs round-robin, and a frame's range starts at a multiple
// of kXcds and has avg_groups(tiles) workgroups, so XCD k runs the frame's
// workgroups k, k + kXcds, ... in order; it gets the k-th run of
// ceil(tiles / kXcds) tiles in strip-major order. Vertically adjacent tiles
// of a strip share 2r rows of every coefficient plane, which then stay in
// that XCD's L2. False for the padding workgroups.
__device__ __forceinline__ bool avg_tile_xcd(int b, int tiles_x, int n_seg, int* sx, int* sy) {
  const int tiles = tiles_x * n_seg;
  const int m = (tiles + kXcds - 1) / kXcds;
  const int t = (b % kXcds) * m + b / kXcds;
  if (t >= tiles) return false;
  *sx = t / n_seg;
  *sy = t - *sx * n_seg;
  return true;
}

template <int Q, int C, int AV, bool BATCH = false>
__global__ void __launch_bounds__(kThreads, kAvgPerCU) apply_avg_kernel(LaunchArgs ain) {
  int bid = blockIdx.x;
  const LaunchArgs a = BATCH ? batch_frame(ain, &bid) : ain;
  int sx, sy;
  if (!avg_tile_xcd(bid, a.tiles_x, a.n_seg, &sx, &sy)) return;  // padding
  apply_avg_tile_any<Q, C, AV>(a, sx, sy);
}

}  // namespace flr

#include "flr_adjoint.hpp"
#include "flr_box.hpp"
#include "flr_lowres.hpp"

namespace flr {

// ---------------------------------------------------------------------------
// The persistent batch kernel (see BatchStage). Thread 0 takes the next item
// and waits for what it depends on; the workgroup runs the item's tile
// function; finished items bump their counter after a release fence. The
// last workgroup to leave resets the queue and the counters for the next
// run (no clearing launch, nothing recorded into a graph but this kernel).
// Waits until *c >= need; gives up (false) after kBatchSpinLimit sleeps, or
// at once when an earlier wait of the run has given up (*failed set), so
// that a broken run ends instead of waiting once per item.
__device__ __forceinline__ bool batch_wait(const int* c, int need, const int* failed) {
  for (int k = 0; k < kBatchSpinLimit; ++k) {
    if (__hip_atomic_load(c, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= need) return true;
    if (__hip_atomic_load(failed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    __builtin_amdgcn_s_sleep(2);
  }
  return false;
}

template <int Q, int C, bool WIDE, int AV>
__global__ void __launch_bounds__(kThreads, 1) batch_kernel(LaunchArgs ain) {
  const BatchPlanDev* P = ain.bplan;
  __shared__ int s_item, s_stage;
  for (;;) {
    __syncthreads();  // the previous item is done with LDS and s_item
    if (threadIdx.x == 0) {
      const int it = atomicAdd(&P->ctl[0], 1);
      int st = -1;
      if (it < P->nitems)
        for (int k = 0; k < P->nstages; ++k)
          if (it >= P->stages[k].first && it < P->stages[k].first + P->stages[k].count) st = k;
      s_item = it;
      s_stage = st;
      if (st >= 0) {  // dependencies
        const BatchStage& S = P->stages[st];
        const int b = it - S.first;
        bool ok = true;
        if (S.kind == BI_AVG) {
          const LaunchArgs& f = P->largs[S.arg];
          const int y0 = (b / f.tiles_x) * f.seg_rows;
          const int y1 = min(y0 + f.seg_rows, f.H);
          const int s0 = max(y0 - f.r, 0) / S.seg_rows;
          const int s1 = min((min(y1 + f.r, f.H) - 1) / S.seg_rows, S.nseg - 1);
          for (int sg = s0; sg <= s1 && ok; ++sg)
            ok = batch_wait(&P->counters[S.wait + sg], S.need, &P->ctl[2]);
        } else if (S.wait >= 0) {
          ok = batch_wait(&P->counters[S.wait], S.need, &P->ctl[2]);
        }
        if (!ok) atomicOr(&P->ctl[2], 1);
      }
    }
    __syncthreads();
    // uniform across the workgroup: scalar registers
    const int st = __builtin_amdgcn_readfirstlane(s_stage);
    if (st < 0) break;
    // every lane sees the writes the item depends on
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const BatchStage S = P->stages[st];
    const int b = __builtin_amdgcn_readfirstlane(s_item) - S.first;
    switch (S.kind) {
      case BI_WALK:
        walk_tile<Q, C, W_COEFFS, WIDE>(P->largs[S.arg], b);
        break;
      case BI_JBOX:
        box_tile_any<BOX_PRODUCTS, WIDE>(P->bargs[S.arg], b % S.nx, b / S.nx);
        break;
      case BI_JSOLVE:
        lr_solve_item<Q, C>(P->largs[S.arg], b);
        break;
      case BI_JMEAN:
        box_tile_any<BOX_MEAN64, WIDE>(P->bargs[S.arg], b % S.nx, b / S.nx);
        break;
      case BI_AVG:
        apply_avg_tile_any<Q, C, AV>(P->largs[S.arg], b % P->largs[S.arg].tiles_x,
                                     b / P->largs[S.arg].tiles_x);
        break;
      default:
        up_apply_item<Q, C>(P->largs[S.arg], b);
        break;
    }
    if (S.done >= 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // this lane's stores
      __syncthreads();
      if (threadIdx.x == 0) {
        const int c = S.kind == BI_WALK ? S.done + b / P->largs[S.arg].tiles_x : S.done;
        __hip_atomic_fetch_add(&P->counters[c], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
  if (threadIdx.x == 0) {
    if (atomicAdd(&P->ctl[1], 1) == (int)gridDim.x - 1) {
      for (int k = 0; k < P->ncounters; ++k) P->counters[k] = 0;
      P->ctl[0] = 0;
      P->ctl[1] = 0;
    }
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

template <typename K>
static hipError_t launch_with_lds_grid(K kernel, dim3 grid, size_t lds, const LaunchArgs& a,
                                       hipStream_t s) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kernel, grid, dim3(kThreads), lds, s, a);
  return hipGetLastError();
}

template <int Q, int C>
hipError_t launch_qc(int kind, const LaunchArgs& a, hipStream_t s) {
  const int64_t pl = (int64_t)a.H * a.W;
  const int pblocks = (int)((pl + 255) / 256);
  const int wblocks = a.tiles_x * a.n_seg;
  const bool wide = wide_segments(a.r);
  const size_t lds = walk_lds_bytes(kind, Q, C);
  auto lds_of = [](int k) { return walk_lds_bytes(k, Q, C); };
  switch (kind) {
    case K_MOMENTS:
      return wide ? launch_with_lds(walk_kernel<Q, C, W_MOMENTS, true>, wblocks, lds, a, s)
                  : launch_with_lds(walk_kernel<Q, C, W_MOMENTS, false>, wblocks, lds, a, s);
    case K_FUSED0:
      return wide ? launch_with_lds(walk_kernel<Q, C, W_FUSED0, true>, wblocks, lds, a, s)
                  : launch_with_lds(walk_kernel<Q, C, W_FUSED0, false>, wblocks, lds, a, s);
    case K_FUSED1:
      return wide ? launch_with_lds(walk_kernel<Q, C, W_FUSED1, true>, wblocks, lds, a, s)
                  : launch_with_lds(walk_kernel<Q, C, W_FUSED1, false>, wblocks, lds, a, s);
    case K_COEFFS:
      return wide ? launch_with_lds(walk_kernel<Q, C, W_COEFFS, true>, wblocks, lds, a, s)
                  : launch_with_lds(walk_kernel<Q, C, W_COEFFS, false>, wblocks, lds, a, s);
    case K_MOMENTS_A:
    case K_MOMENTS_B:
      if constexpr (split_walk(Q, C)) {
        constexpr int PA = split_first(Q, C), NPQ = num_products(Q, C);
        if (kind == K_MOMENTS_A) {
          const size_t l2 = walk_lds_bytes(K_MOMENTS, Q, C, Q + C + PA);
          return wide ? launch_with_lds(walk_kernel<Q, C, W_MOMENTS, true, 0, PA>, wblocks, l2, a, s)
                      : launch_with_lds(walk_kernel<Q, C, W_MOMENTS, false, 0, PA>, wblocks, l2, a, s);
        }
        const size_t l2 = walk_lds_bytes(K_MOMENTS, Q, C, Q + C + NPQ - PA);
        return wide ? launch_with_lds(walk_kernel<Q, C, W_MOMENTS, true, PA, NPQ - PA>, wblocks, l2, a, s)
                    : launch_with_lds(walk_kernel<Q, C, W_MOMENTS, false, PA, NPQ - PA>, wblocks, l2, a, s);
      }
      return hipErrorInvalidValue;
    case K_SPLIT_COEFFS:
      if constexpr (split_walk(Q, C)) {
        constexpr int PA = split_first(Q, C), NPQ = num_products(Q, C);
        const size_t l2 = walk_lds_bytes(K_COEFFS, Q, C, Q + C + NPQ - PA);
        return wide ? launch_with_lds(walk_kernel<Q, C, W_SPLITSOLVE, true, PA, NPQ - PA>,
                                      wblocks, l2, a, s)
                    : launch_with_lds(walk_kernel<Q, C, W_SPLITSOLVE, false, PA, NPQ - PA>,
                                      wblocks, l2, a, s);
      }
      return hipErrorInvalidValue;
    case K_APPLY_AVG:
      switch (avg_variant(a.r, C)) {
        case AV_BLOCK8:
          if constexpr (C <= 3)
            return launch_with_lds(apply_avg_kernel<Q, C, AV_BLOCK8>, avg_groups(wblocks), lds, a,
                                   s);
          return hipErrorInvalidValue;
        case AV_STREAM64:
          return launch_with_lds(apply_avg_kernel<Q, C, AV_STREAM64>, avg_groups(wblocks), lds, a,
                                 s);
        default:
          return launch_with_lds(apply_avg_kernel<Q, C, AV_STREAM16>, avg_groups(wblocks), lds, a,
                                 s);
      }
    case K_SOLVE:
      hipLaunchKernelGGL((solve_kernel<Q, C>), dim3(pblocks), dim3(256), 0, s, a);
      return hipGetLastError();
    case K_APPLY_POINT:
      hipLaunchKernelGGL((apply_point_kernel<Q, C>), dim3(pblocks), dim3(256), 0, s, a);
      return hipGetLastError();
    case K_ADJ_COEF:
      hipLaunchKernelGGL((adj_coef_kernel<Q, C>), dim3(pblocks), dim3(256), 0, s, a);
      return hipGetLastError();
    case K_ADJ_SOLVE:
      hipLaunchKernelGGL((adj_solve_kernel<Q, C>), dim3(pblocks), dim3(256), 0, s, a);
      return hipGetLastError();
    case K_ADJ_GATHER:
      hipLaunchKernelGGL((adj_gather_kernel<Q, C>), dim3(pblocks), dim3(256), 0, s, a);
      return hipGetLastError();
    case K_LR_BLOCK: {
      const int nx = (a.W + kThreads - 1) / kThreads;
      hipLaunchKernelGGL((lr_block_kernel<Q, C>), dim3(nx, a.Hl), dim3(kThreads), 0, s, a);
      return hipGetLastError();
    }
    case K_LR_SOLVE: {
      const int lb = (int)(((int64_t)a.Hl * a.Wl + 255) / 256);
      hipLaunchKernelGGL((lr_solve_kernel<Q, C>), dim3(lb), dim3(256), 0, s, a);
      return hipGetLastError();
    }
    case K_COEFFS_BATCH:
      if constexpr (!split_walk(Q, C)) {
        return wide ? launch_with_lds(walk_kernel<Q, C, W_COEFFS, true, 0, -1, true>,
                                      a.batch_blocks, lds_of(K_COEFFS), a, s)
                    : launch_with_lds(walk_kernel<Q, C, W_COEFFS, false, 0, -1, true>,
                                      a.batch_blocks, lds_of(K_COEFFS), a, s);
      }
      return hipErrorInvalidValue;
    case K_APPLY_AVG_BATCH:
      switch (avg_variant(a.r, C)) {
        case AV_BLOCK8:
          if constexpr (C <= 3)
            return launch_with_lds(apply_avg_kernel<Q, C, AV_BLOCK8, true>, a.batch_blocks,
                                   lds_of(K_APPLY_AVG), a, s);
          return hipErrorInvalidValue;
        case AV_STREAM64:
          return launch_with_lds(apply_avg_kernel<Q, C, AV_STREAM64, true>, a.batch_blocks,
                                 lds_of(K_APPLY_AVG), a, s);
        default:
          return launch_with_lds(apply_avg_kernel<Q, C, AV_STREAM16, true>, a.batch_blocks,
                                 lds_of(K_APPLY_AVG), a, s);
      }
    case K_UP_APPLY_BATCH:
      hipLaunchKernelGGL((up_apply_kernel<Q, C, true>), dim3(a.batch_blocks), dim3(256), 0, s, a);
      return hipGetLastError();
    case K_BATCH_PERSISTENT:
      if constexpr (!split_walk(Q, C)) {
        const size_t l = batch_lds_bytes(Q, C);
        const int av = avg_variant(a.r, C);
        if (av == AV_BLOCK8) {
          if constexpr (C <= 3) return launch_with_lds(batch_kernel<Q, C, false, AV_BLOCK8>,
                                                       a.batch_blocks, l, a, s);
          return hipErrorInvalidValue;
        }
        if (av == AV_STREAM64)
          return launch_with_lds(batch_kernel<Q, C, true, AV_STREAM64>, a.batch_blocks, l, a, s);
        return launch_with_lds(batch_kernel<Q, C, false, AV_STREAM16>, a.batch_blocks, l, a, s);
      }
      return hipErrorInvalidValue;
    case K_LR_APPLY:
      if (a.lr_rows > 0) {
        const size_t l = lr_apply_lds_bytes(Q, C, a.block, a.lr_rows);
        const dim3 grid((a.W + kThreads - 1) / kThreads, (a.H + a.lr_rows - 1) / a.lr_rows);
        return launch_with_lds_grid(lr_apply_staged_kernel<Q, C>, grid, l, a, s);
      }
      hipLaunchKernelGGL((lr_apply_kernel<Q, C>), dim3(pblocks), dim3(256), 0, s, a);
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
