// Adjoint of the FLR path (reverse-mode gradients of flr_denoise), one lane
// per pixel, templated on (Q, C). Included by flr_device.hpp after the
// regulariser and Cholesky helpers.
//
// Forward, per pixel k with clipped window T_k of n_k pixels (Sec. 3.1-3.2,
// Appendix): window means mu (guides), nu (noisy), central moments
// W = (1/n) sum (g - mu)(g - mu)^T and V = (1/n) sum (g - mu)(y - nu)^T, the
// regularised system H(W, mu; eps, eps') a = V, b = nu - a^T mu; optionally
// abar_i = (1/n_i) sum_{k in T_i} a_k (and bbar); out_i = bbar_i + abar_i^T g_i.
//
// Reverse, given G_i = dL/d(out_i):
//   averaging   A_k = dL/da_k = sum_{i in T_k} g_i G_i^T / n_i, B_k = dL/db_k =
//               sum_{i in T_k} G_i / n_i (windows are symmetric: i in T_k iff
//               k in T_i); without averaging A_k = g_k G_k^T, B_k = G_k. The
//               direct term dL/dg_i gets abar_i G_i.
//   intercept   b = nu - a^T mu: dnu = B, dmu = -a B, A' = A - mu B^T.
//   solve       a = H^-1 V: Gv = dL/dV = H^-1 A' (H symmetric), dL/dH has the
//               symmetric part Gs = -(Gv a^T + a Gv^T) / 2.
//   regulariser ridge H = W + eps I: dW = Gs, dL/deps += tr Gs.
//               Appendix H = W^ + eps diag(W^), W^ = W + eps'(mu mu^T +
//               diag(mu o mu)) + eps I: dW^ = Gs with its diagonal times
//               (1 + eps); dL/deps += sum_q Gs_qq W^_qq + tr dW^; dL/deps' +=
//               mu^T dW^ mu + sum_q dW^_qq mu_q^2; dmu += 2 eps'(dW^ mu +
//               diag(dW^) o mu); dW = dW^.
//   moments     with sum (g - mu) = 0 over the window the mean terms drop:
//               dL/dg_j += sum_{k in T_j} (1/n_k) [2 dW_k (g_j - mu_k) +
//               Gv_k (y_j - nu_k) + dmu_k], dL/dy_j += sum_{k in T_j} (1/n_k)
//               [Gv_k^T (g_j - mu_k) + dnu_k].
// The last line is evaluated as window sums of per-pixel fields
//   O_k = 2 dW_k / n_k, Gam_k = Gv_k / n_k,
//   e_k = (dmu_k - 2 dW_k mu_k - Gv_k nu_k) / n_k, f_k = (dnu_k - Gv_k^T mu_k) / n_k,
// contracted at the pixel: dL/dg_j = (sum O) g_j + (sum Gam) y_j + sum e,
// dL/dy_j = (sum Gam)^T g_j + sum f.
//
// Precision: every g and y above may be shifted by a constant per plane
// (sum (g - mu) = 0 makes the result shift-free), so all of it runs on
// inputs anchored at their value at pixel (0, 0), in FP64: moments from
// FP64 window sums of the anchored products (not the FP32 moment planes,
// whose rounded means would enter the cancelling differences g - mu and
// A - mu B^T), FP64 fields and FP64 window sums. Only the Appendix
// regulariser sees the original-unit means.
#pragma once

namespace flr {

// Anchors: each input plane's value at pixel (0, 0).
template <int Q, int C>
__device__ __forceinline__ void load_anchors(const LaunchArgs& a, int64_t pl, double (&cg)[Q],
                                             double (&cy)[C]) {
#pragma unroll
  for (int q = 0; q < Q; ++q) cg[q] = a.guides[q * pl];
#pragma unroll
  for (int c = 0; c < C; ++c) cy[c] = a.noisy[c * pl];
}

// Anchored window means mu~, nu~, the central moments W (upper triangle)
// and V from the raw sums of the anchored products, channel ch (moment
// order g | y | g g^T upper | g y^T) read as sum(ch).
template <int Q, int C, typename F>
__device__ __forceinline__ void centred_from(F&& sum, double inv_n, double (&mu)[Q],
                                             double (&nu)[C], double (&Hm)[Q * (Q + 1) / 2],
                                             double* V, int vstride) {
  constexpr int NP = Q * (Q + 1) / 2;
#pragma unroll
  for (int q = 0; q < Q; ++q) mu[q] = sum(q) * inv_n;
#pragma unroll
  for (int c = 0; c < C; ++c) nu[c] = sum(Q + c) * inv_n;
#pragma unroll
  for (int p = 0; p < Q; ++p) {
#pragma unroll
    for (int q = p; q < Q; ++q)
      Hm[tri<Q>(p, q)] = fma(sum(Q + C + tri<Q>(p, q)), inv_n, -mu[p] * mu[q]);
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
#pragma unroll
    for (int c = 0; c < C; ++c)
      V[q * vstride + c] = fma(sum(Q + C + NP + q * C + c), inv_n, -mu[q] * nu[c]);
  }
}

// The same from FP64 sum planes [num_sums][H][W] at pixel S.
template <int Q, int C>
__device__ __forceinline__ void centred_moments(const double* S, int64_t pl, double inv_n,
                                                double (&mu)[Q], double (&nu)[C],
                                                double (&Hm)[Q * (Q + 1) / 2], double* V,
                                                int vstride) {
  centred_from<Q, C>([&](int ch) { return S[ch * pl]; }, inv_n, mu, nu, Hm, V, vstride);
}

// Coefficients a of pixel j (FP64, from the moment sums), a.fout [Q*C]: with
// averaging their window sums give n abar (the window sums of the averaging
// products G_c / n_j and g~_q G_c / n_j, which give B and A~, are formed from
// the inputs by the window-sum pass); without averaging A~ and B are formed
// where needed and a is read back.
template <int Q, int C>
__global__ void __launch_bounds__(256) adj_coef_kernel(LaunchArgs a) {
  using T = double;
  constexpr int NP = Dims<Q, C>::NP;
  const int64_t pl = (int64_t)a.H * a.W;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= pl) return;
  const int i = (int)(idx / a.W), j = (int)(idx - (int64_t)i * a.W);
  const T inv_n = T(1) / (T)(win_count(i, a.H, a.r) * win_count(j, a.W, a.r));
  T cg[Q], cy[C];
  load_anchors<Q, C>(a, pl, cg, cy);
  T mu[Q], nu[C], Hm[NP], R[Q * C], mo[Q];
  centred_moments<Q, C>(a.sums + idx, pl, inv_n, mu, nu, Hm, R, C);
#pragma unroll
  for (int q = 0; q < Q; ++q) mo[q] = mu[q] + cg[q];
  regularise<Q, T>(Hm, mo, (T)arg_eps(a), (T)arg_eps_mul(a), a.reg_mode);
  chol_solve<Q, C, T>(Hm, R);
  double* o = a.fout + idx;
#pragma unroll
  for (int k = 0; k < Q * C; ++k) o[k * pl] = R[k];
}

// Solve adjoint of pixel k from its moment sums (a.sums) and A~, B (window
// sums of the averaging fields in a.fin, or formed from g~ and G without
// averaging) -> the fields O, Gam, e, f in anchored units (a.fout) and this
// workgroup's sums of dL/deps and dL/deps' (a.red).
template <int Q, int C>
__global__ void __launch_bounds__(256) adj_solve_kernel(LaunchArgs a) {
  using T = double;
  constexpr int NP = Dims<Q, C>::NP;
  constexpr int C2 = 2 * C;
  __shared__ double part[2][kThreads];
  const int tid = threadIdx.x;
  const int64_t pl = (int64_t)a.H * a.W;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + tid;
  T de = 0, dm = 0;
  if (idx < pl) {
    const int i = (int)(idx / a.W), j = (int)(idx - (int64_t)i * a.W);
    const T inv_n = T(1) / (T)(win_count(i, a.H, a.r) * win_count(j, a.W, a.r));
    T cg[Q], cy[C];
    load_anchors<Q, C>(a, pl, cg, cy);
    // R columns: V (-> a), then A' = A~ - mu~ B^T (-> Gv)
    T mu[Q], nu[C], Hm[NP], R[Q * C2], B[C], mo[Q];
    centred_moments<Q, C>(a.sums + idx, pl, inv_n, mu, nu, Hm, R, C2);
    bool clamped[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      clamped[q] = Hm[tri<Q>(q, q)] < T(0);
      mo[q] = mu[q] + cg[q];
    }
    // A~ and B: window sums of the averaging fields, or formed at the pixel
    // (two wave-uniform paths, each with its loads issued together)
    T A[Q * C];
    if (a.average) {
#pragma unroll
      for (int c = 0; c < C; ++c) B[c] = a.fin[c * pl + idx];
#pragma unroll
      for (int k = 0; k < Q * C; ++k) A[k] = a.fin[(C + k) * pl + idx];
    } else {
      T gq[Q];
#pragma unroll
      for (int c = 0; c < C; ++c) B[c] = a.gout[c * pl + idx];
#pragma unroll
      for (int q = 0; q < Q; ++q) gq[q] = (T)a.guides[q * pl + idx] - cg[q];
#pragma unroll
      for (int k = 0; k < Q * C; ++k) A[k] = gq[k / C] * B[k % C];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
#pragma unroll
      for (int c = 0; c < C; ++c) R[q * C2 + C + c] = fma(-mu[q], B[c], A[q * C + c]);
    }
    regularise<Q, T>(Hm, mo, (T)arg_eps(a), (T)arg_eps_mul(a), a.reg_mode);
    T hd[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) hd[q] = Hm[tri<Q>(q, q)];
    chol_solve<Q, C2, T>(Hm, R);
    // R[q][c] = a_qc, R[q][C + c] = Gv_qc
    T dmu[Q], dW[NP];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      T s = 0;
#pragma unroll
      for (int c = 0; c < C; ++c) s = fma(R[q * C2 + c], B[c], s);
      dmu[q] = -s;
    }
#pragma unroll
    for (int p = 0; p < Q; ++p) {
#pragma unroll
      for (int q = p; q < Q; ++q) {
        T s = 0;
#pragma unroll
        for (int c = 0; c < C; ++c)
          s = fma(R[p * C2 + C + c], R[q * C2 + c], fma(R[p * C2 + c], R[q * C2 + C + c], s));
        dW[tri<Q>(p, q)] = T(-0.5) * s;
      }
    }
    if (a.reg_mode == 0) {
#pragma unroll
      for (int q = 0; q < Q; ++q) de += dW[tri<Q>(q, q)];
    } else {
      const T eps = arg_eps(a), em = arg_eps_mul(a), s1 = T(1) + eps;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        de = fma(dW[tri<Q>(q, q)], hd[q] / s1, de);  // Gs_qq W^_qq
        dW[tri<Q>(q, q)] *= s1;                       // dW^
        de += dW[tri<Q>(q, q)];
      }
#pragma unroll
      for (int p = 0; p < Q; ++p) {
        T s = 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) s = fma(dW[tri<Q>(p < q ? p : q, p < q ? q : p)], mo[q], s);
        const T dpp = dW[tri<Q>(p, p)];
        dm = fma(mo[p], s, dm);
        dm = fma(dpp * mo[p], mo[p], dm);
        dmu[p] = fma(T(2) * em, fma(dpp, mo[p], s), dmu[p]);
      }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
      if (clamped[q]) dW[tri<Q>(q, q)] = T(0);
    double* o = a.fout + idx;
#pragma unroll
    for (int k = 0; k < NP; ++k) o[k * pl] = T(2) * dW[k] * inv_n;
#pragma unroll
    for (int k = 0; k < Q * C; ++k) o[(NP + k) * pl] = R[(k / C) * C2 + C + k % C] * inv_n;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
      T s = dmu[p];
#pragma unroll
      for (int q = 0; q < Q; ++q)
        s = fma(T(-2) * dW[tri<Q>(p < q ? p : q, p < q ? q : p)], mu[q], s);
#pragma unroll
      for (int c = 0; c < C; ++c) s = fma(-R[p * C2 + C + c], nu[c], s);
      o[(NP + Q * C + p) * pl] = s * inv_n;
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      T s = B[c];
#pragma unroll
      for (int q = 0; q < Q; ++q) s = fma(-R[q * C2 + C + c], mu[q], s);
      o[(NP + Q * C + Q + c) * pl] = s * inv_n;
    }
  }
  // fixed-order workgroup sums of the regulariser gradients
  part[0][tid] = de;
  part[1][tid] = dm;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (tid < s) {
      part[0][tid] += part[0][tid + s];
      part[1][tid] += part[1][tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    a.red[2 * blockIdx.x] = part[0][0];
    a.red[2 * blockIdx.x + 1] = part[1][0];
  }
}

// dL/dg and dL/dy of pixel j: the window sums of the solve fields (a.fin)
// contracted with the anchored g~_j, y~_j, plus abar_j G_j with abar the
// window sums of a (a.fin2, Q*C planes) divided by n_j, or a itself without
// averaging.
template <int Q, int C>
__global__ void __launch_bounds__(256) adj_gather_kernel(LaunchArgs a) {
  using T = double;
  constexpr int NP = Dims<Q, C>::NP;
  const int64_t pl = (int64_t)a.H * a.W;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= pl) return;
  const int i = (int)(idx / a.W), j = (int)(idx - (int64_t)i * a.W);
  const T scale = a.average ? T(1) / (T)(win_count(i, a.H, a.r) * win_count(j, a.W, a.r)) : T(1);
  T cg[Q], cy[C];
  load_anchors<Q, C>(a, pl, cg, cy);
  T g[Q], y[C], G[C];
#pragma unroll
  for (int q = 0; q < Q; ++q) g[q] = (T)a.guides[q * pl + idx] - cg[q];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    y[c] = (T)a.noisy[c * pl + idx] - cy[c];
    G[c] = a.gout[c * pl + idx];
  }
  const double* S = a.fin + idx;
  const double* Ab = a.fin2 + idx;
#pragma unroll
  for (int p = 0; p < Q; ++p) {
    T s = S[(NP + Q * C + p) * pl];
#pragma unroll
    for (int q = 0; q < Q; ++q) s = fma(S[tri<Q>(p < q ? p : q, p < q ? q : p) * pl], g[q], s);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      s = fma(S[(NP + p * C + c) * pl], y[c], s);
      s = fma(Ab[(p * C + c) * pl] * scale, G[c], s);
    }
    a.out[p * pl + idx] = (float)s;
  }
#pragma unroll
  for (int c = 0; c < C; ++c) {
    T s = S[(NP + Q * C + Q + c) * pl];
#pragma unroll
    for (int q = 0; q < Q; ++q) s = fma(S[(NP + q * C + c) * pl], g[q], s);
    a.out2[c * pl + idx] = (float)s;
  }
}

}  // namespace flr
