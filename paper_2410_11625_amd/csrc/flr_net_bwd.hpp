// Gradients of the FLNR guide network (Sec. 3.3 trains the network by
// backpropagating the loss through the regression into it).
//
// Straight-through reading of the BF16 network: the backward treats every
// BF16 rounding of the forward as the identity, so the gradients are those of
// the exact network evaluated at the BF16 weights and activations the forward
// produced. All backward arithmetic is FP32; gradients between layers are FP32
// HWC tensors ([pixel][channel]).
//
//   ReLU layer      dz = g * [a > 0], a the stored BF16 activation (a > 0
//                   exactly when the FP32 pre-activation is > 0: BF16 keeps
//                   the FP32 exponent range)
//   sigmoid head    dz = g * s (1 - s), s the FP32 output
//   conv            db[o] = sum_q dz[q][o]
//                   dW[o][c][u][v] = sum_(i,j) dz[(i,j)][o] x[(s i + u - p, s j + v - p)][c]
//                   dx[(y,x)][c] = sum_(o,u,v) W[o][c][u][v] dz[((y + p - u)/s, (x + p - v)/s)][o]
//                   over the terms whose division is exact and in range
//   up2 + concat    the coarse tensor collects the gradients of the 2x2 fine
//                   pixels that copied it; the skip takes its channels as is
//
// Weight gradients reduce over every output pixel: each workgroup sums one
// pixel chunk into a partial, and a second kernel adds the chunks in a fixed
// order, so the result does not depend on scheduling.

namespace flrnet {

constexpr int kWgOB = 4;  // output channels per weight-gradient entry
constexpr int kWgCB = 8;  // input channels per weight-gradient entry
constexpr int kWgAcc = kWgOB * kWgCB;

// wr[i] = BF16 rounding of p[i] (the weights the forward multiplies by).
struct RoundArgs {
  const float* p;
  float* wr;
  int n;
};
__global__ void __launch_bounds__(256) round_params_kernel(RoundArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.n) a.wr[i] = bf2f(f2bf(a.p[i]));
}

// dz[q][o] = dout[o][q] s (1 - s), s = sig[o][q] (planar in, HWC out).
struct SigmoidBwdArgs {
  const float* dout;
  const float* sig;
  float* dz;
  int npx, nout;
};
__global__ void __launch_bounds__(256) sigmoid_bwd_kernel(SigmoidBwdArgs a) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.npx) return;
  for (int o = 0; o < a.nout; ++o) {
    const float s = a.sig[(size_t)o * a.npx + q];
    a.dz[(size_t)q * a.nout + o] = a.dout[(size_t)o * a.npx + q] * s * (1.f - s);
  }
}

// Input of a layer as the backward reads it: one HWC BF16 tensor, or
// [up2(in0), in1] with in0 on a grid of width Wl (Wl = 0: plain).
struct BwdSrc {
  const uint16_t* in0;
  const uint16_t* in1;
  int cs0, cup, cs1;  // in0 channel stride, channels taken from in0, in1 channel stride
  int Wl;
};

// Eight input channels c0..c0+7 (c0 % 8 == 0) at input pixel (yi, xi), which
// the caller has clamped into the grid.
__device__ __forceinline__ void load_x8(const BwdSrc& s, int Wi, int yi, int xi, int c0,
                                        float (&x)[kWgCB]) {
  const uint16_t* p;
  if (s.Wl > 0 && c0 < s.cup)
    p = s.in0 + ((size_t)(yi >> 1) * s.Wl + (xi >> 1)) * s.cs0 + c0;
  else if (s.Wl > 0)
    p = s.in1 + ((size_t)yi * Wi + xi) * s.cs1 + (c0 - s.cup);
  else
    p = s.in0 + ((size_t)yi * Wi + xi) * s.cs0 + c0;
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    x[2 * k] = __uint_as_float(w[k] << 16);
    x[2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
  }
}

// dz at output pixel q, channels o..o+3: the output gradient, masked by the
// stored ReLU activation when act is given.
__device__ __forceinline__ float4 load_dz4(const float* g, const uint16_t* act, size_t q, int cout,
                                           int o) {
  float4 d = *reinterpret_cast<const float4*>(g + q * cout + o);
  if (act) {
    const uint2 a = *reinterpret_cast<const uint2*>(act + q * cout + o);
    d.x = (a.x & 0xffffu) != 0 && !(a.x & 0x8000u) ? d.x : 0.f;
    d.y = (a.x >> 16) != 0 && !(a.x & 0x80000000u) ? d.y : 0.f;
    d.z = (a.y & 0xffffu) != 0 && !(a.y & 0x8000u) ? d.z : 0.f;
    d.w = (a.y >> 16) != 0 && !(a.y & 0x80000000u) ? d.w : 0.f;
  }
  return d;
}

struct WgradArgs {
  const float* g;       // [Ho*Wo][cout] gradient of the layer's output activation
  const uint16_t* act;  // [Ho*Wo][cout] stored activation (ReLU mask), or null
  BwdSrc src;
  int Hi, Wi, Ho, Wo;
  int cout, ncb, k, stride;  // ncb: 8-channel blocks of the stored input
  int ne;                    // entries: (cout / 4) * ncb * k * k
  int chunk_px;              // output pixels per chunk (blockIdx.x)
  float* part;               // [nchunk][ne * 32 + cout]: entries' sums, then the bias sums
};

// One wave per row of KW taps (kernel row u) of 4 output channels x 8 input
// channels: entries e0 .. e0 + KW - 1 with e0 = ((ob ncb + cb) k + u) k.
// The 64 lanes stride over a chunk of output pixels, loading dz once for the
// row's taps; the lanes' sums are added in LDS in lane order, one tap at a
// time.
template <int KW>
__global__ void __launch_bounds__(256) wgrad_kernel(WgradArgs a) {
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int kk = KW * KW;
  const int nrow = a.ne / KW;
  const int w = blockIdx.y * 4 + wave;
  const bool live = w < nrow;
  const int u = live ? w % KW : 0;
  const int cb = live ? (w / KW) % a.ncb : 0;
  const int ob = live ? w / KW / a.ncb : 0;
  const int e0 = ((ob * a.ncb + cb) * KW + u) * KW;
  const int pd = KW / 2;
  const bool with_bias = live && cb == 0 && u == 0;
  float acc[KW][kWgAcc];
  float bacc[kWgOB];
#pragma unroll
  for (int v = 0; v < KW; ++v)
#pragma unroll
    for (int i = 0; i < kWgAcc; ++i) acc[v][i] = 0.f;
#pragma unroll
  for (int i = 0; i < kWgOB; ++i) bacc[i] = 0.f;
  const size_t npx = (size_t)a.Ho * a.Wo;
  const size_t q0 = (size_t)blockIdx.x * a.chunk_px;
  const size_t q1 = q0 + a.chunk_px < npx ? q0 + a.chunk_px : npx;
  if (live) {
    for (size_t q = q0 + lane; q < q1; q += 64) {
      const int i = (int)(q / a.Wo), j = (int)(q % a.Wo);
      const int yi = a.stride * i + u - pd;
      const bool oky = yi >= 0 && yi < a.Hi;
      const int yc = yi < 0 ? 0 : (yi >= a.Hi ? a.Hi - 1 : yi);
      float x[KW][kWgCB];
#pragma unroll
      for (int v = 0; v < KW; ++v) {
        const int xi = a.stride * j + v - pd;
        const bool ok = oky && xi >= 0 && xi < a.Wi;
        const int xc = xi < 0 ? 0 : (xi >= a.Wi ? a.Wi - 1 : xi);
        load_x8(a.src, a.Wi, yc, xc, cb * kWgCB, x[v]);
#pragma unroll
        for (int c = 0; c < kWgCB; ++c) x[v][c] = ok ? x[v][c] : 0.f;
      }
      const float4 d4 = load_dz4(a.g, a.act, q, a.cout, ob * kWgOB);
      const float d[kWgOB] = {d4.x, d4.y, d4.z, d4.w};
#pragma unroll
      for (int o = 0; o < kWgOB; ++o) {
        bacc[o] += d[o];
#pragma unroll
        for (int v = 0; v < KW; ++v)
#pragma unroll
          for (int c = 0; c < kWgCB; ++c) acc[v][o * kWgCB + c] += d[o] * x[v][c];
      }
    }
  }
  constexpr int kRow = kWgAcc + kWgOB + 1;  // + 1: staggers the LDS banks
  float* red = flr::lds + wave * 64 * kRow;
  float* row = a.part + (size_t)blockIdx.x * (a.ne * kWgAcc + a.cout);
#pragma unroll
  for (int v = 0; v < KW; ++v) {
    if (v > 0) __syncthreads();  // the previous tap's sums have been read
#pragma unroll
    for (int i = 0; i < kWgAcc; ++i) red[lane * kRow + i] = acc[v][i];
#pragma unroll
    for (int i = 0; i < kWgOB; ++i) red[lane * kRow + kWgAcc + i] = bacc[i];
    __syncthreads();
    if (live && lane < kWgAcc + kWgOB) {
      float s = 0.f;
      for (int l = 0; l < 64; ++l) s += red[l * kRow + lane];
      if (lane < kWgAcc)
        row[(e0 + v) * kWgAcc + lane] = s;
      else if (with_bias && v == 0)
        row[a.ne * kWgAcc + ob * kWgOB + (lane - kWgAcc)] = s;
    }
  }
}
constexpr size_t wgrad_lds_bytes() { return 4 * 64 * (kWgAcc + kWgOB + 1) * sizeof(float); }

// First level of the chunk sum: out[g][slot] = sum of in[ch][slot] over
// the chunks ch of group g (kChunkGroup consecutive chunks), in order.
constexpr int kChunkGroup = 32;
struct ChunkSumArgs {
  const float* in;
  float* out;
  int S, nchunk;
};
__global__ void __launch_bounds__(256) chunk_sum_kernel(ChunkSumArgs a) {
  const int ng = (a.nchunk + kChunkGroup - 1) / kChunkGroup;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)ng * a.S) return;
  const int g = (int)(idx / a.S), slot = (int)(idx % a.S);
  const int c0 = g * kChunkGroup;
  const int c1 = c0 + kChunkGroup < a.nchunk ? c0 + kChunkGroup : a.nchunk;
  float s = 0.f;
  for (int ch = c0; ch < c1; ++ch) s += a.in[(size_t)ch * a.S + slot];
  a.out[idx] = s;
}

struct WreduceArgs {
  const float* part;  // [nchunk][ne * 32 + cout]
  int nchunk, ne, ncb, cin, cout, k;
  float* grad;  // the layer's weights [cout][cin][k][k] then bias [cout]
  int accumulate;
};

// grad = (accumulate ? grad : 0) + the chunk partials, added in chunk order.
// One thread per partial slot (entry e, slot j), so the chunk loop reads
// consecutive addresses across the wave; the result goes to its weight.
__global__ void __launch_bounds__(256) wreduce_kernel(WreduceArgs a) {
  const int kk = a.k * a.k;
  const int np = a.ne * kWgAcc, S = np + a.cout;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= S) return;
  int dst;
  if (idx < np) {
    const int e = idx / kWgAcc, j = idx % kWgAcc;
    const int tap = e % kk, cb = (e / kk) % a.ncb, ob = e / kk / a.ncb;
    const int o = ob * kWgOB + j / kWgCB, c = cb * kWgCB + j % kWgCB;
    if (c >= a.cin) return;  // padding channels of the stored input
    dst = (o * a.cin + c) * kk + tap;
  } else {
    dst = a.cout * a.cin * kk + (idx - np);
  }
  float s = 0.f;
  for (int ch = 0; ch < a.nchunk; ++ch) s += a.part[(size_t)ch * S + idx];
  a.grad[dst] = a.accumulate ? a.grad[dst] + s : s;
}

struct DgradArgs {
  const float* g;       // [Ho*Wo][cout]
  const uint16_t* act;  // ReLU mask or null
  const float* w;       // BF16-rounded weights [cout][cin][k][k]
  int cin, cout, k, stride;
  int Hi, Wi, Ho, Wo;
  float* dx;            // [Hi*Wi][cin]
  const float* add;     // optional addend add[p * add_cs + add_off + c]
  int add_cs, add_off;
};

// One thread per input pixel and kDgC input channels (blockIdx.y picks
// them); the workgroup first stages those channels' weights in LDS as
// [tap][o][kDgC]. 16 channels halve the dz loads per multiply-add; 8 give
// twice the workgroups, which small frames need to fill the chip.
template <int kDgC>
__global__ void __launch_bounds__(256) dgrad_kernel(DgradArgs a) {
  float* wl = flr::lds;
  const int c0 = blockIdx.y * kDgC;
  const int pd = a.k / 2, kk = a.k * a.k;
  const int nw = kk * a.cout * kDgC;
  for (int t = threadIdx.x; t < nw; t += blockDim.x) {
    const int c = t % kDgC, o = (t / kDgC) % a.cout, tap = t / (kDgC * a.cout);
    wl[t] = a.w[((size_t)o * a.cin + c0 + c) * kk + tap];
  }
  __syncthreads();
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t npx = (size_t)a.Hi * a.Wi;
  if (p >= npx) return;
  const int y = (int)(p / a.Wi), x = (int)(p % a.Wi);
  float acc[kDgC];
#pragma unroll
  for (int c = 0; c < kDgC; ++c) acc[c] = 0.f;
  for (int u = 0; u < a.k; ++u) {
    const int ny = y + pd - u;
    if (ny < 0 || ny % a.stride) continue;
    const int i = ny / a.stride;
    if (i >= a.Ho) continue;
    for (int v = 0; v < a.k; ++v) {
      const int nx = x + pd - v;
      if (nx < 0 || nx % a.stride) continue;
      const int j = nx / a.stride;
      if (j >= a.Wo) continue;
      const size_t q = (size_t)i * a.Wo + j;
      const float* wt = wl + (size_t)(u * a.k + v) * a.cout * kDgC;
      for (int o = 0; o < a.cout; o += 4) {
        const float4 d4 = load_dz4(a.g, a.act, q, a.cout, o);
        const float d[4] = {d4.x, d4.y, d4.z, d4.w};
#pragma unroll
        for (int oo = 0; oo < 4; ++oo) {
#pragma unroll
          for (int c4 = 0; c4 < kDgC; c4 += 4) {
            const float4 w4 = *reinterpret_cast<const float4*>(wt + (o + oo) * kDgC + c4);
            acc[c4 + 0] += w4.x * d[oo];
            acc[c4 + 1] += w4.y * d[oo];
            acc[c4 + 2] += w4.z * d[oo];
            acc[c4 + 3] += w4.w * d[oo];
          }
        }
      }
    }
  }
  float* dst = a.dx + p * a.cin + c0;
  if (a.add) {
    const float* ad = a.add + p * a.add_cs + a.add_off + c0;
#pragma unroll
    for (int c = 0; c < kDgC; ++c) dst[c] = acc[c] + ad[c];
  } else {
#pragma unroll
    for (int c = 0; c < kDgC; ++c) dst[c] = acc[c];
  }
}
inline size_t dgrad_lds_bytes(const Layer& L, int cpt) {
  return (size_t)L.k * L.k * L.cout * cpt * sizeof(float);
}
// grids from 2^18 pixels take 16 channels per thread (the sum order per
// channel is the same either way; a build may lower the threshold)
#ifndef FLR_DGRAD_WIDE_PX
#define FLR_DGRAD_WIDE_PX (1 << 18)
#endif
constexpr size_t kDgWidePx = (size_t)(FLR_DGRAD_WIDE_PX);

// low[(i,j)][c] = sum of fine[(2i+di, 2j+dj)][c] over the fine pixels in the
// H x W grid, channels c < nc of a fine tensor with channel stride cs.
struct Up2BwdArgs {
  const float* fine;
  int H, W, cs;
  float* low;
  int Hl, Wl, nc;
};
__global__ void __launch_bounds__(256) up2_bwd_kernel(Up2BwdArgs a) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)a.Hl * a.Wl * a.nc) return;
  const int c = (int)(idx % a.nc);
  const size_t pl = idx / a.nc;
  const int i = (int)(pl / a.Wl), j = (int)(pl % a.Wl);
  float s = 0.f;
  for (int di = 0; di < 2; ++di)
    for (int dj = 0; dj < 2; ++dj) {
      const int y = 2 * i + di, x = 2 * j + dj;
      if (y < a.H && x < a.W) s += a.fine[((size_t)y * a.W + x) * a.cs + c];
    }
  a.low[idx] = s;
}

// Chunking of a weight-gradient launch: about kWgTarget workgroups (4 per
// CU), chunks of whole waves of pixels and at least kWgMinIters pixels per
// lane, so that the pixel loop outweighs the wave's closing LDS reduction.
constexpr int kWgTarget = 2048;
constexpr int kWgMinIters = 16;
struct WgradPlan {
  int ne, wg_y, chunk_px, nchunk;
};
inline WgradPlan wgrad_plan(const Layer& L, int ncb, size_t npx) {
  WgradPlan p;
  p.ne = (L.cout / kWgOB) * ncb * L.k * L.k;
  p.wg_y = (p.ne / L.k + 3) / 4;  // one wave per row of L.k taps
  const size_t waves = (npx + 63) / 64;
  size_t want = (kWgTarget + p.wg_y - 1) / p.wg_y;
  if (want > (waves + kWgMinIters - 1) / kWgMinIters) want = (waves + kWgMinIters - 1) / kWgMinIters;
  if (want < 1) want = 1;
  const size_t per = (waves + want - 1) / want;
  p.chunk_px = (int)(per * 64);
  p.nchunk = (int)((npx + p.chunk_px - 1) / p.chunk_px);
  return p;
}
inline int stored_cin_blocks(int li) { return li == 0 ? 2 : kLayers[li].cin / kWgCB; }

}  // namespace flrnet
