// The paper's fast FLR variant (Sec. 3.2): the moment tensor downsampled by
// B x B block sums, a small Gaussian blur at the low resolution, one
// regularised solve per low-resolution pixel, and the models bilinearly
// interpolated back to full resolution, where they are applied. Kernels
// templated on (Q, C); included by flr_device.hpp after the adjoint, whose
// centred-moment helper it shares.
//
// Precision: the block sums, the blur and the solve are FP64 on inputs
// anchored at their value at pixel (0, 0) (moments and models are shift-
// free; the Appendix regulariser alone sees the original-unit means). The
// models are kept in anchored units, b~ = nu~ - a^T mu~, and applied as
// out = (b~ + anchor_y) + a^T (g - anchor_g).
#pragma once

namespace flr {

// Factors of moment channel ch (order g | y | g g^T upper | g y^T): input
// planes u and v of the concatenated guides and noisy channels, v = -1 for
// a first moment.
struct ChanUV {
  int u, v;
};
template <int Q, int C>
__host__ __device__ constexpr ChanUV chan_uv(int ch) {
  if (ch < Q + C) return {ch, -1};
  ch -= Q + C;
  if (ch < Q * (Q + 1) / 2) {
    int p = 0;
    while (ch >= Q - p) {
      ch -= Q - p;
      ++p;
    }
    return {p, p + ch};
  }
  ch -= Q * (Q + 1) / 2;
  return {ch / C, Q + ch % C};
}

// Block sums. Lane l of a workgroup owns input column blockIdx.x * kThreads
// + l over the B rows of low-resolution row blockIdx.y and sums the anchored
// products of that column in FP64 registers (loads issued four rows at a
// time); the B lanes of each block then add their sums with DPP butterflies
// inside their 16-lane row (quad_perm xor 1 and xor 2, row_half_mirror,
// row_mirror: every lane of the block ends with the block sum), and the
// block's first lane writes it. More channels than fit in registers are
// taken in equal chunks, each re-reading the inputs.
constexpr int kLrMaxAcc = 80;
constexpr int kDppXor1 = 0xB1;       // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;       // quad_perm [2, 3, 0, 1]
constexpr int kDppRowMirror = 0x140;
constexpr int kDppRowHalfMirror = 0x141;

// Sum over aligned groups of B (1, 2, 4, 8 or 16) lanes, in every lane of
// the group. Every lane of the wavefront must take part.
// The moves always run and the block size only selects which are added, so
// the sums of many channels can be interleaved without branches.
__device__ __forceinline__ double group_sum(double v, int B) {
  double m = dpp_move<kDppXor1, 0xf>(v);
  v += B >= 2 ? m : 0.0;
  m = dpp_move<kDppXor2, 0xf>(v);
  v += B >= 4 ? m : 0.0;
  m = dpp_move<kDppRowHalfMirror, 0xf>(v);
  v += B >= 8 ? m : 0.0;
  m = dpp_move<kDppRowMirror, 0xf>(v);
  v += B >= 16 ? m : 0.0;
  return v;
}

template <int Q, int C>
__global__ void __launch_bounds__(256) lr_block_kernel(LaunchArgs a) {
  constexpr int NS = num_sums(Q, C);
  constexpr int NV = Q + C;
  constexpr int NCHUNK = (NS + kLrMaxAcc - 1) / kLrMaxAcc;
  constexpr int CH = (NS + NCHUNK - 1) / NCHUNK;
  const int tid = threadIdx.x;
  const int B = a.block;
  const int64_t pl = (int64_t)a.H * a.W;
  const int64_t pll = (int64_t)a.Hl * a.Wl;
  const int x = blockIdx.x * kThreads + tid;
  const int I = blockIdx.y;
  const int y0 = I * B;
  const int y1 = y0 + B < a.H ? y0 + B : a.H;
  const bool inx = x < a.W;
  const int J = blockIdx.x * (kThreads / B) + tid / B;
  const bool writer = (tid % B) == 0 && J < a.Wl;
  double anc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) anc[v] = v < Q ? a.guides[v * pl] : a.noisy[(v - Q) * pl];
  const int64_t col = inx ? x : 0;
  static_for<0, NCHUNK>([&](auto K) {
    constexpr int k0 = decltype(K)::value * CH;
    constexpr int kn = NS - k0 < CH ? NS - k0 : CH;
    double acc[kn];
#pragma unroll
    for (int l = 0; l < kn; ++l) acc[l] = 0.0;
    for (int yb = y0; yb < y1; yb += 4) {
      // unconditional loads (rows past the block repeat its last row and
      // are dropped below), so that all of them are in flight together
      float zf[4][NV];
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int y = yb + rr < y1 ? yb + rr : y1 - 1;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const float* src = v < Q ? a.guides + v * pl : a.noisy + (v - Q) * pl;
          zf[rr][v] = src[(int64_t)y * a.W + col];
        }
      }
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        if (yb + rr >= y1) break;
        double z[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) z[v] = inx ? (double)zf[rr][v] - anc[v] : 0.0;
        static_for<0, kn>([&](auto L) {
          constexpr int l = decltype(L)::value;
          constexpr ChanUV uv = chan_uv<Q, C>(k0 + l);
          if constexpr (uv.v < 0)
            acc[l] += z[uv.u];
          else
            acc[l] = fma(z[uv.u], z[uv.v], acc[l]);
        });
      }
    }
#pragma unroll
    for (int l = 0; l < kn; ++l) {
      const double s = group_sum(acc[l], B);
      if (writer) a.fout[(1 + k0 + l) * pll + (int64_t)I * a.Wl + J] = s;
    }
  });
  if (writer) {
    const int x1 = (J + 1) * B < a.W ? (J + 1) * B : a.W;
    a.fout[(int64_t)I * a.Wl + J] = (double)((y1 - y0) * (x1 - J * B));
  }
}

// Regularised solve of each low-resolution pixel from the blurred planes
// (a.fin: count, then the channel sums) -> models b~ (C), a (Q*C) in a.fout.
template <int Q, int C>
__device__ __forceinline__ void lr_solve_item(const LaunchArgs a, const int bid) {
  using T = double;
  constexpr int NP = Dims<Q, C>::NP;
  const int64_t pll = (int64_t)a.Hl * a.Wl;
  const int64_t idx = (int64_t)bid * 256 + threadIdx.x;
  if (idx >= pll) return;
  const int64_t pl = (int64_t)a.H * a.W;
  const double* S = a.fin + idx;
  const T inv_n = T(1) / S[0];
  T mu[Q], nu[C], Hm[NP], R_[Q * C], mo[Q];
  centred_from<Q, C>([&](int ch) { return S[(1 + ch) * pll]; }, inv_n, mu, nu, Hm, R_, C);
#pragma unroll
  for (int q = 0; q < Q; ++q) mo[q] = mu[q] + (T)a.guides[q * pl];
  regularise<Q, T>(Hm, mo, (T)arg_eps(a), (T)arg_eps_mul(a), a.reg_mode);
  chol_solve<Q, C, T>(Hm, R_);
  double* o = a.fout + idx;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    T b = nu[c];
#pragma unroll
    for (int q = 0; q < Q; ++q) b = fma(-R_[q * C + c], mu[q], b);
    o[c * pll] = b;
  }
#pragma unroll
  for (int k = 0; k < Q * C; ++k) o[(C + k) * pll] = R_[k];
}
template <int Q, int C>
__global__ void __launch_bounds__(256) lr_solve_kernel(LaunchArgs a) {
  lr_solve_item<Q, C>(a, blockIdx.x);
}

// Bilinear interpolation of the models at each full-resolution pixel
// (half-pixel centres: low-resolution coordinate (i + 0.5) / B - 0.5,
// clamped to the grid) and reconstruction.
template <int Q, int C>
__global__ void __launch_bounds__(256) lr_apply_kernel(LaunchArgs a) {
  using T = double;
  const int64_t pl = (int64_t)a.H * a.W;
  const int64_t pll = (int64_t)a.Hl * a.Wl;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= pl) return;
  const int i = (int)(idx / a.W), j = (int)(idx - (int64_t)i * a.W);
  auto axis = [&](int k, int n_low, int* k0, int* k1, T* t) {
    T u = ((T)k + T(0.5)) / (T)a.block - T(0.5);
    u = u < T(0) ? T(0) : (u > (T)(n_low - 1) ? (T)(n_low - 1) : u);
    const int f = (int)u;  // u >= 0
    *k0 = f;
    *k1 = f + 1 < n_low ? f + 1 : n_low - 1;
    *t = u - (T)f;
  };
  int r0, r1, c0, c1;
  T tr, tc;
  axis(i, a.Hl, &r0, &r1, &tr);
  axis(j, a.Wl, &c0, &c1, &tc);
  const int64_t o00 = (int64_t)r0 * a.Wl + c0, o01 = (int64_t)r0 * a.Wl + c1;
  const int64_t o10 = (int64_t)r1 * a.Wl + c0, o11 = (int64_t)r1 * a.Wl + c1;
  auto model = [&](int k) {
    const double* m = a.fin + k * pll;
    const T top = m[o00] * (T(1) - tc) + m[o01] * tc;
    const T bot = m[o10] * (T(1) - tc) + m[o11] * tc;
    return top * (T(1) - tr) + bot * tr;
  };
  T g[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) g[q] = (T)a.guides[q * pl + idx] - (T)a.guides[q * pl];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    T s = model(c) + (T)a.noisy[c * pl];
#pragma unroll
    for (int q = 0; q < Q; ++q) s = fma(model(C + q * C + c), g[q], s);
    a.out[c * pl + idx] = (float)s;
  }
}

// Low-resolution coordinate of full-resolution index k: half-pixel centres,
// clamped to [0, n_low - 1]; neighbours k0, k1 and the weight of k1.
__device__ __forceinline__ void lr_axis(int k, int block, int n_low, int* k0, int* k1,
                                        double* t) {
  double u = ((double)k + 0.5) / (double)block - 0.5;
  u = u < 0.0 ? 0.0 : (u > (double)(n_low - 1) ? (double)(n_low - 1) : u);
  const int f = (int)u;
  *k0 = f;
  *k1 = f + 1 < n_low ? f + 1 : n_low - 1;
  *t = u - (double)f;
}

// The same as lr_apply_kernel with the vertical half of the interpolation
// done once per workgroup: a workgroup covers a.lr_rows full-resolution rows
// by kThreads columns; it first stages, for each of its rows, the models
// interpolated between the two low-resolution rows at every low-resolution
// column its pixels use ([row][model][column] in LDS), then each lane
// interpolates along its row from two staged columns and applies the model.
template <int Q, int C>
__global__ void __launch_bounds__(256) lr_apply_staged_kernel(LaunchArgs a) {
  using T = double;
  constexpr int FC = (Q + 1) * C;
  extern __shared__ float lds[];
  double* st = reinterpret_cast<double*>(lds);
  const int tid = threadIdx.x;
  const int64_t pl = (int64_t)a.H * a.W;
  const int64_t pll = (int64_t)a.Hl * a.Wl;
  const int X0 = blockIdx.x * kThreads;
  const int Y0 = blockIdx.y * a.lr_rows;
  const int TR = a.lr_rows;
  const int xl = X0 + kThreads - 1 < a.W - 1 ? X0 + kThreads - 1 : a.W - 1;
  int c_lo, c_hi, d0, d1;
  double dt;
  lr_axis(X0, a.block, a.Wl, &c_lo, &d0, &dt);
  lr_axis(xl, a.block, a.Wl, &d1, &c_hi, &dt);
  const int nc = c_hi - c_lo + 1;
  // staging, kStage items per lane at a time: the loads of a batch are
  // issued together (items past the end repeat the last one, unstored)
  constexpr int kStage = 8;
  const int total = TR * FC * nc;
  for (int t0 = 0; t0 < total; t0 += kStage * kThreads) {
    double v0[kStage], v1[kStage], w[kStage];
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      int t = t0 + u * kThreads + tid;
      t = t < total ? t : total - 1;
      const int rr = t / (FC * nc);
      const int rem = t - rr * (FC * nc);
      const int k = rem / nc, cc = rem - (rem / nc) * nc;
      const int y = Y0 + rr < a.H ? Y0 + rr : a.H - 1;
      int r0, r1;
      lr_axis(y, a.block, a.Hl, &r0, &r1, &w[u]);
      const double* m = a.fin + k * pll + c_lo + cc;
      v0[u] = m[(int64_t)r0 * a.Wl];
      v1[u] = m[(int64_t)r1 * a.Wl];
    }
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      const int t = t0 + u * kThreads + tid;
      if (t < total) st[t] = v0[u] * (T(1) - w[u]) + v1[u] * w[u];
    }
  }
  __syncthreads();
  const int x = X0 + tid;
  if (x >= a.W) return;
  int c0, c1;
  double tc;
  lr_axis(x, a.block, a.Wl, &c0, &c1, &tc);
  c0 -= c_lo;
  c1 -= c_lo;
  T anc_g[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) anc_g[q] = a.guides[q * pl];
  for (int rr = 0; rr < TR; ++rr) {
    const int y = Y0 + rr;
    if (y >= a.H) break;
    const int64_t idx = (int64_t)y * a.W + x;
    const double* row = st + rr * FC * nc;
    auto model = [&](int k) { return row[k * nc + c0] * (T(1) - tc) + row[k * nc + c1] * tc; };
    T g[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) g[q] = (T)a.guides[q * pl + idx] - anc_g[q];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      T s = model(c) + (T)a.noisy[c * pl];
#pragma unroll
      for (int q = 0; q < Q; ++q) s = fma(model(C + q * C + c), g[q], s);
      a.out[c * pl + idx] = (float)s;
    }
  }
}

// Joint denoising and upsampling (Sec. 3.2): anchored FP64 models (b~ | a,
// as lr_solve_kernel writes them, window-averaged) on a grid a.Hl x a.Wl,
// a.up times coarser than the output, bilinearly interpolated at each output
// pixel (half-pixel centres, clamped) and applied to the full-resolution
// guides with the anchors of the fit (pixel (0, 0) of the low-resolution
// guides and of the noisy input). Batched over frames.
template <int Q, int C>
__device__ __forceinline__ void up_apply_item(const LaunchArgs a, const int bid) {
  using T = double;
  constexpr int FC = (Q + 1) * C;
  const int64_t pl = (int64_t)a.H * a.W;
  const int64_t pll = (int64_t)a.Hl * a.Wl;
  const int64_t idx = (int64_t)bid * 256 + threadIdx.x;
  if (idx >= pl) return;
  const int i = (int)(idx / a.W), j = (int)(idx - (int64_t)i * a.W);
  int r0, r1, c0, c1;
  double tr, tc;
  lr_axis(i, a.up, a.Hl, &r0, &r1, &tr);
  lr_axis(j, a.up, a.Wl, &c0, &c1, &tc);
  const int64_t o00 = (int64_t)r0 * a.Wl + c0, o01 = (int64_t)r0 * a.Wl + c1;
  const int64_t o10 = (int64_t)r1 * a.Wl + c0, o11 = (int64_t)r1 * a.Wl + c1;
  T m[FC];
#pragma unroll
  for (int k = 0; k < FC; ++k) {
    const double* p = a.fin + k * pll;
    const T top = p[o00] * (T(1) - tc) + p[o01] * tc;
    const T bot = p[o10] * (T(1) - tc) + p[o11] * tc;
    m[k] = top * (T(1) - tr) + bot * tr;
  }
  T g[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) g[q] = (T)a.guides[q * pl + idx] - (T)a.guides_low[q * pll];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    T s = m[c] + (T)a.noisy[c * pll];
#pragma unroll
    for (int q = 0; q < Q; ++q) s = fma(m[C + q * C + c], g[q], s);
    a.out[c * pl + idx] = (float)s;
  }
}
template <int Q, int C, bool BATCH>
__global__ void __launch_bounds__(256) up_apply_kernel(LaunchArgs ain) {
  int bid = blockIdx.x;
  const LaunchArgs a = BATCH ? batch_frame(ain, &bid) : ain;
  up_apply_item<Q, C>(a, bid);
}

}  // namespace flr
