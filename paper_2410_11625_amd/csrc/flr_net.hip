// The FLNR guide network (Sec. 3.3, the three-level 16/32/64 variant
// declared in include/flr_net.h) on the gfx950 matrix cores, and FLNR
// denoising (network, then FLR over the 12 guides).
//
// Every layer is one implicit-GEMM kernel. Activations are BF16 in HWC order
// (channels innermost, a multiple of 16), so the 16 channels of one K step
// of a pixel are 32 contiguous bytes. With A = weights (c_out x k) and
// B = input (k x pixels), v_mfma_f32_16x16x16_bf16 gives lane l the
// accumulators of output channels 4*(l/16) .. +3 of pixel l % 16: four
// consecutive channels, stored as one 8-byte write, and exactly the B
// operand layout of a following 1x1 layer, which is therefore fused into the
// producing kernel (in3 + in1, out3 + out1). Upsampling and concatenation
// are folded into the consumer's operand loads. A workgroup of four waves
// covers 64 consecutive output pixels of one row, each wave 16 pixels and
// all output channels; weights are packed once into the per-lane fragment
// order, so each A operand is one contiguous 512-byte read per wave.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include "flr.h"
#include "flr_net.h"

// The workgroup's dynamic LDS (one array shared by every kernel of the library).
namespace flr {
extern __shared__ float lds[];
}

namespace flrnet {

typedef short bf16x4_t __attribute__((vector_size(8)));
typedef float f32x4_t __attribute__((vector_size(16)));

enum InKind : int { IN_HWC = 0, IN_UPCAT = 2 };
enum Fuse : int { FUSE_NONE = 0, FUSE_1X1_RELU = 1, FUSE_1X1_SIGMOID = 2 };

struct ConvArgs {
  const uint16_t* in0;  // HWC BF16 input (IN_UPCAT: the low-resolution part)
  const uint16_t* in1;  // IN_UPCAT: the skip connection, on the conv's input grid
  const bf16x4_t* w;    // packed weight fragments of the layer
  const float* b;       // BF16-rounded bias (padded output channels)
  const bf16x4_t* w2;   // fused 1x1 layer
  const float* b2;
  uint16_t* out;        // HWC BF16 output
  float* outf;          // FUSE_1X1_SIGMOID: planar FP32 output
  uint16_t* mid;        // fused layers: when set, the first layer's BF16
                        // activations are stored here too (HWC, 16 channels)
  int Hi, Wi;           // input grid
  int Hl, Wl;           // IN_UPCAT: grid of in0
  int Ho, Wo;           // output grid
};

// FP32 -> BF16, round to nearest, ties to even (NaN stays NaN).
__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x4_t pack4(uint16_t a, uint16_t b, uint16_t c, uint16_t d) {
  bf16x4_t v;
  v[0] = (short)a;
  v[1] = (short)b;
  v[2] = (short)c;
  v[3] = (short)d;
  return v;
}

// Four consecutive input channels c..c+3 of input pixel (yi, xi), which
// the caller has clamped into the input grid; the caller zeroes padding.
// CB: the 16-channel block (compile-time, so the source choice folds);
// c4 = 4 * (lane / 16), the lane's channel quad within the block.
template <int CIN, int CUP, int IN, int CB>
__device__ __forceinline__ bf16x4_t load_in(const ConvArgs& a, int yi, int xi, int c4) {
  constexpr int c0 = CB * 16;
  if constexpr (IN == IN_UPCAT && c0 < CUP)
    return *reinterpret_cast<const bf16x4_t*>(a.in0 + ((size_t)(yi >> 1) * a.Wl + (xi >> 1)) * CUP +
                                              c0 + c4);
  else if constexpr (IN == IN_UPCAT)
    return *reinterpret_cast<const bf16x4_t*>(a.in1 + ((size_t)yi * a.Wi + xi) * (CIN - CUP) +
                                              (c0 - CUP) + c4);
  else
    return *reinterpret_cast<const bf16x4_t*>(a.in0 + ((size_t)yi * a.Wi + xi) * CIN + c0 + c4);
}

// All NCB channel blocks of one input pixel (zero where !ok).
template <int CIN, int CUP, int IN, int NCB, int CB = 0>
__device__ __forceinline__ void load_blocks(const ConvArgs& a, int yi, int xi, int c4, bool ok,
                                            bf16x4_t (&dst)[NCB]) {
  if constexpr (CB < NCB) {
    const bf16x4_t v = load_in<CIN, CUP, IN, CB>(a, yi, xi, c4);
    dst[CB] = ok ? v : pack4(0, 0, 0, 0);
    load_blocks<CIN, CUP, IN, NCB, CB + 1>(a, yi, xi, c4, ok, dst);
  }
}

// Network input: the 8 guides and 3 noisy planes (planar FP32) of one pixel,
// each compressed to sign(v) log(1 + |v|), rounded to BF16 and written as
// one HWC row of 16 channels (the last 5 zero).
struct PrepArgs {
  const float* g;
  const float* y;
  uint16_t* out;
  int H, W;
};
__global__ void __launch_bounds__(256) prep_kernel(PrepArgs a) {
  const size_t pl = (size_t)a.H * a.W;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= pl) return;
  uint16_t h[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    float v = 0.f;
    if (c < FLR_NET_IN_GUIDES) v = a.g[c * pl + i];
    else if (c < FLR_NET_IN_GUIDES + FLR_NET_IN_NOISY) v = a.y[(c - FLR_NET_IN_GUIDES) * pl + i];
    h[c] = f2bf(copysignf(log1pf(fabsf(v)), v));
  }
  bf16x4_t* o = reinterpret_cast<bf16x4_t*>(a.out + i * 16);
#pragma unroll
  for (int q = 0; q < 4; ++q) o[q] = pack4(h[4 * q], h[4 * q + 1], h[4 * q + 2], h[4 * q + 3]);
}

// One conv layer (CIN, COUT multiples of 16; KS 1 or 3; stride ST), bias and
// ReLU, optionally followed by a fused 1x1 layer to COUT2 channels (ReLU to
// HWC BF16, or sigmoid to planar FP32).
// Bias, ReLU and store of one tile (lane l: channels 4*(l/16)..+3 of each
// 16-channel block, pixel px), or the fused 1x1 layer on those activations.
template <int COUT, int FUSE, int COUT2>
__device__ __forceinline__ void epilogue(const ConvArgs& a, int y, int px, bool pin, int kq,
                                         int lane, const f32x4_t (&acc)[COUT / 16]) {
  constexpr int NB = COUT / 16;
  if constexpr (FUSE == FUSE_NONE) {
    if (!pin) return;
    uint16_t* o = a.out + ((size_t)y * a.Wo + px) * COUT + 4 * kq;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      uint16_t h[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) h[i] = f2bf(fmaxf(acc[nb][i] + a.b[nb * 16 + 4 * kq + i], 0.f));
      *reinterpret_cast<bf16x4_t*>(o + nb * 16) = pack4(h[0], h[1], h[2], h[3]);
    }
  } else {
    static_assert(COUT == 16, "a fused 1x1 layer reads 16 channels");
    // this layer's activations are the B operand of the 1x1 layer as they are
    uint16_t h[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) h[i] = f2bf(fmaxf(acc[0][i] + a.b[4 * kq + i], 0.f));
    const bf16x4_t hv = pack4(h[0], h[1], h[2], h[3]);
    if (a.mid && pin)
      *reinterpret_cast<bf16x4_t*>(a.mid + ((size_t)y * a.Wo + px) * 16 + 4 * kq) = hv;
    constexpr int NB2 = (COUT2 + 15) / 16;
#pragma unroll
    for (int nb = 0; nb < NB2; ++nb) {
      f32x4_t d = f32x4_t{0.f, 0.f, 0.f, 0.f};
      d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.w2[nb * 64 + lane], hv, d, 0, 0, 0);
      if (!pin) continue;
      if (FUSE == FUSE_1X1_RELU) {
        uint16_t q[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) q[i] = f2bf(fmaxf(d[i] + a.b2[nb * 16 + 4 * kq + i], 0.f));
        *reinterpret_cast<bf16x4_t*>(a.out + ((size_t)y * a.Wo + px) * COUT2 + nb * 16 + 4 * kq) =
            pack4(q[0], q[1], q[2], q[3]);
      } else {
        const size_t pl = (size_t)a.Ho * a.Wo, off = (size_t)y * a.Wo + px;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = nb * 16 + 4 * kq + i;
          if (c < COUT2) a.outf[c * pl + off] = 1.f / (1.f + expf(-(d[i] + a.b2[c])));
        }
      }
    }
  }
}

// DPP lane move of an 8-byte fragment within 16-lane rows (two 32-bit moves).
constexpr int kDppRowShl1 = 0x101, kDppRowShr1 = 0x111, kDppRowRor1 = 0x121,
              kDppRowRor15 = 0x12F;
template <int CTRL>
__device__ __forceinline__ bf16x4_t dpp_frag(bf16x4_t v) {
  int w[2];
  __builtin_memcpy(w, &v, sizeof w);
  w[0] = __builtin_amdgcn_update_dpp(0, w[0], CTRL, 0xf, 0xf, true);
  w[1] = __builtin_amdgcn_update_dpp(0, w[1], CTRL, 0xf, 0xf, true);
  bf16x4_t r;
  __builtin_memcpy(&r, w, sizeof w);
  return r;
}

// Four tiles of 16 output pixels per wave: the input fragments of the four
// tiles for one kernel row are in flight together and each weight fragment
// is reused across them.
__host__ __device__ constexpr int tiles_per_wave(int) { return 4; }

template <int CIN, int COUT, int KS, int ST, int IN, int CUP, int FUSE, int COUT2>
__global__ void __launch_bounds__(256) conv_kernel(ConvArgs a) {
  constexpr int NCB = CIN / 16, NB = COUT / 16, P = KS / 2, TPW = tiles_per_wave(CIN);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int y = blockIdx.y;
  const int kq = lane >> 4;
  int px[TPW];
  bool pin[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    px[t] = (blockIdx.x * 4 + wv) * TPW * 16 + t * 16 + (lane & 15);
    pin[t] = px[t] < a.Wo;
  }
  // partial sums (K steps round-robin) so that at least 8 independent MFMA
  // chains are in flight per wave
  constexpr int KSPL = (TPW * NB >= 8) ? 1 : 8 / (TPW * NB);
  f32x4_t acc[TPW][NB][KSPL];
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int k = 0; k < KSPL; ++k) acc[t][nb][k] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ky = 0; ky < KS; ++ky) {
    const int yi = y * ST + ky - P;
    const bool oky = yi >= 0 && yi < a.Hi;
    const int yc = min(max(yi, 0), a.Hi - 1);
    // this kernel row's input fragments of every tile, then their products
    bf16x4_t bv[TPW][KS][NCB];
    if constexpr (ST == 1 && KS == 3) {
      // Only the centre column (kx = 1) of each tile and one pixel beyond
      // each end of the four tiles are loaded. In the B layout a 16-lane DPP
      // row holds 16 consecutive pixels of one channel group, so kx = 0 is
      // the centre shifted right by one lane (row_shr) with lane 0 taking
      // lane 15 of the tile before (row_ror:1), and kx = 2 the centre shifted
      // left (row_shl) with lane 15 taking lane 0 of the next tile
      // (row_ror:15). Out-of-image pixels are zero in the centre and halo
      // loads, hence in every shifted copy.
      bf16x4_t hl[NCB], hr[NCB];
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int xc = min(max(px[t], 0), a.Wi - 1);
        load_blocks<CIN, CUP, IN, NCB>(a, yc, xc, 4 * kq, pin[t] && oky, bv[t][1]);
      }
      {
        const int xl = px[0] - 1, xr = px[TPW - 1] + 1;
        load_blocks<CIN, CUP, IN, NCB>(a, yc, min(max(xl, 0), a.Wi - 1), 4 * kq,
                                       oky && xl >= 0 && xl < a.Wi, hl);
        load_blocks<CIN, CUP, IN, NCB>(a, yc, min(max(xr, 0), a.Wi - 1), 4 * kq,
                                       oky && xr >= 0 && xr < a.Wi, hr);
      }
      const bool first = (lane & 15) == 0, last = (lane & 15) == 15;
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          const bf16x4_t left = t == 0 ? hl[cb] : dpp_frag<kDppRowRor1>(bv[t - 1][1][cb]);
          const bf16x4_t shr = dpp_frag<kDppRowShr1>(bv[t][1][cb]);
          bv[t][0][cb] = first ? left : shr;
          const bf16x4_t right = t == TPW - 1 ? hr[cb] : dpp_frag<kDppRowRor15>(bv[t + 1][1][cb]);
          const bf16x4_t shl = dpp_frag<kDppRowShl1>(bv[t][1][cb]);
          bv[t][2][cb] = last ? right : shl;
        }
      }
    } else if constexpr (ST == 2 && KS == 3 && CIN <= 32) {
      // Stride 2: kx = 1 and kx = 2 read input pixels 2p and 2p + 1; kx = 0
      // reads 2p - 1, the kx = 2 pixel of the lane before (row_shr), lane 0
      // taking lane 15 of the tile before (row_ror:1) or, for the first
      // tile, one loaded halo pixel. (Measured: faster at 32 input channels,
      // slower at 64, where the three loads per tile are kept.)
      bf16x4_t hl[NCB];
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
#pragma unroll
        for (int kx = 1; kx < 3; ++kx) {
          const int xi = px[t] * 2 + kx - 1;
          const int xc = min(max(xi, 0), a.Wi - 1);
          load_blocks<CIN, CUP, IN, NCB>(a, yc, xc, 4 * kq, pin[t] && oky && xi < a.Wi,
                                         bv[t][kx]);
        }
      }
      {
        const int xl = px[0] * 2 - 1;
        load_blocks<CIN, CUP, IN, NCB>(a, yc, min(max(xl, 0), a.Wi - 1), 4 * kq,
                                       oky && xl >= 0 && xl < a.Wi, hl);
      }
      const bool first = (lane & 15) == 0;
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          const bf16x4_t left = t == 0 ? hl[cb] : dpp_frag<kDppRowRor1>(bv[t - 1][2][cb]);
          const bf16x4_t shr = dpp_frag<kDppRowShr1>(bv[t][2][cb]);
          bv[t][0][cb] = first ? left : shr;
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
#pragma unroll
        for (int kx = 0; kx < KS; ++kx) {
          const int xi = px[t] * ST + kx - P;
          const bool ok = pin[t] && oky && xi >= 0 && xi < a.Wi;
          const int xc = min(max(xi, 0), a.Wi - 1);
          load_blocks<CIN, CUP, IN, NCB>(a, yc, xc, 4 * kq, ok, bv[t][kx]);
        }
      }
    }
#pragma unroll
    for (int kx = 0; kx < KS; ++kx) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int tap = ky * KS + kx;
        const int ks = (tap * NCB + cb) % KSPL;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const bf16x4_t av = a.w[((tap * NCB + cb) * NB + nb) * 64 + lane];
#pragma unroll
          for (int t = 0; t < TPW; ++t)
            acc[t][nb][ks] =
                __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv[t][kx][cb], acc[t][nb][ks], 0, 0, 0);
        }
      }
    }
  }
  f32x4_t sum[TPW][NB];
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      sum[t][nb] = acc[t][nb][0];
#pragma unroll
      for (int k = 1; k < KSPL; ++k) sum[t][nb] += acc[t][nb][k];
    }
#pragma unroll
  for (int t = 0; t < TPW; ++t) epilogue<COUT, FUSE, COUT2>(a, y, px[t], pin[t], kq, lane, sum[t]);
}

// Stride-1 3x3 layers, input tile in LDS. A workgroup computes kTileRows
// output rows (one per wave) of kTilePx pixels (four tiles of 16) for all
// output channels. It first stages the (kTileRows + 2) x (kTilePx + 2) input
// pixels of the tile with all their channels in LDS (HWC, 8-byte chunks,
// zero outside the image; the decoder's upsampling and concatenation happen
// here), so each input row is fetched by 1.5 output rows instead of 3, and
// the MFMA B fragments are then read from LDS. The MFMA sequence is that of
// conv_kernel, so the two give identical results.
constexpr int kTileRows = 4, kTilePx = 64;
constexpr int kStRows = kTileRows + 2, kStPx = kTilePx + 2;
__host__ __device__ constexpr size_t conv_tile_lds_bytes(int cin) {
  return (size_t)kStRows * kStPx * cin * sizeof(uint16_t);
}

template <int CIN, int COUT, int IN, int CUP, int FUSE, int COUT2>
__global__ void __launch_bounds__(256) conv_tile_kernel(ConvArgs a) {
  constexpr int NCB = CIN / 16, NB = COUT / 16, TPW = 4, KS = 3;
  constexpr int CQ = CIN / 4;                   // 8-byte chunks per pixel
  constexpr int NCH = kStRows * kStPx * CQ;     // chunks to stage
  bf16x4_t* st = reinterpret_cast<bf16x4_t*>(flr::lds);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, kq = lane >> 4;
  const int x0 = blockIdx.x * kTilePx, y0 = blockIdx.y * kTileRows;
  for (int b0 = 0; b0 < NCH; b0 += 8 * 256) {
    bf16x4_t v[8];
    bool ok[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = b0 + u * 256 + tid;
      const int ic = i < NCH ? i : NCH - 1;
      const int pix = ic / CQ, c = 4 * (ic - pix * CQ);
      const int sr = pix / kStPx, sx = pix - sr * kStPx;
      const int yi = y0 - 1 + sr, xi = x0 - 1 + sx;
      ok[u] = i < NCH && yi >= 0 && yi < a.Hi && xi >= 0 && xi < a.Wi;
      const int yc = min(max(yi, 0), a.Hi - 1), xc = min(max(xi, 0), a.Wi - 1);
      const uint16_t* src;
      if constexpr (IN == IN_UPCAT) {
        // one load from a selected address: the upsampled coarse half or the skip
        // (both addresses in range: the unused one's channel is clamped)
        const int cl = c < CUP ? c : CUP - 4, ch = c < CUP ? 0 : c - CUP;
        const uint16_t* lo = a.in0 + ((size_t)(yc >> 1) * a.Wl + (xc >> 1)) * CUP + cl;
        const uint16_t* hi = a.in1 + ((size_t)yc * a.Wi + xc) * (CIN - CUP) + ch;
        src = c < CUP ? lo : hi;
      } else {
        src = a.in0 + ((size_t)yc * a.Wi + xc) * CIN + c;
      }
      v[u] = *reinterpret_cast<const bf16x4_t*>(src);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = b0 + u * 256 + tid;
      if (i < NCH) st[i] = ok[u] ? v[u] : pack4(0, 0, 0, 0);
    }
  }
  __syncthreads();
  const int y = y0 + wv;
  if (y >= a.Ho) return;  // uniform across the wave; no barrier follows
  int px[TPW];
  bool pin[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    px[t] = x0 + t * 16 + (lane & 15);
    pin[t] = px[t] < a.Wo;
  }
  constexpr int KSPL = (TPW * NB >= 8) ? 1 : 8 / (TPW * NB);
  f32x4_t acc[TPW][NB][KSPL];
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int k = 0; k < KSPL; ++k) acc[t][nb][k] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ky = 0; ky < KS; ++ky) {
#pragma unroll
    for (int kx = 0; kx < KS; ++kx) {
      bf16x4_t bv[TPW][NCB];
#pragma unroll
      for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
          bv[t][cb] = st[((wv + ky) * kStPx + t * 16 + (lane & 15) + kx) * CQ + cb * 4 + kq];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int tap = ky * KS + kx;
        const int ks = (tap * NCB + cb) % KSPL;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const bf16x4_t av = a.w[((tap * NCB + cb) * NB + nb) * 64 + lane];
#pragma unroll
          for (int t = 0; t < TPW; ++t)
            acc[t][nb][ks] =
                __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv[t][cb], acc[t][nb][ks], 0, 0, 0);
        }
      }
    }
  }
  f32x4_t sum[TPW][NB];
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      sum[t][nb] = acc[t][nb][0];
#pragma unroll
      for (int k = 1; k < KSPL; ++k) sum[t][nb] += acc[t][nb][k];
    }
#pragma unroll
  for (int t = 0; t < TPW; ++t) epilogue<COUT, FUSE, COUT2>(a, y, px[t], pin[t], kq, lane, sum[t]);
}

// Packing: FP32 weight [cout][cin][k][k] -> fragments (tap, cin block,
// cout block, lane) of 4 BF16, lane l holding output channel 16*nb + l%16
// and input channels 16*cb + 4*(l/16) .. +3; zero in the padding.
struct PackArgs {
  const float* w;  // [cout][cin][ks][ks]
  const float* b;  // [cout]
  int cin, cout, ks, ncb, nb;
  bf16x4_t* wp;    // fragments
  float* bp;       // [16 * nb]
};
__global__ void pack_kernel(PackArgs p) {
  const float* w = p.w;
  const float* b = p.b;
  const int cin = p.cin, cout = p.cout, ks = p.ks, ncb = p.ncb, nb = p.nb;
  bf16x4_t* wp = p.wp;
  float* bp = p.bp;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int nfrag = ks * ks * ncb * nb * 64;
  if (idx < nfrag) {
    const int lane = idx % 64;
    const int n = (idx / 64) % nb;
    const int cb = (idx / 64 / nb) % ncb;
    const int tap = idx / (64 * nb * ncb);
    const int ky = tap / ks, kx = tap % ks;
    const int co = n * 16 + lane % 16;
    uint16_t h[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int ci = cb * 16 + 4 * (lane / 16) + j;
      h[j] = (co < cout && ci < cin) ? f2bf(w[((co * cin + ci) * ks + ky) * ks + kx]) : (uint16_t)0;
    }
    wp[idx] = pack4(h[0], h[1], h[2], h[3]);
  }
  if (idx < nb * 16) bp[idx] = idx < cout ? bf2f(f2bf(b[idx])) : 0.f;
}

// ---------------------------------------------------------------------------
// Host side: layer table, packed-block and workspace layout, launches.

struct Layer {
  int cin, cout, k, stride;
};
constexpr Layer kLayers[12] = {
    {11, 16, 3, 1},  // in3
    {16, 16, 1, 1},  // in1
    {16, 32, 3, 1},  // e1a
    {32, 32, 3, 2},  // e1b
    {32, 64, 3, 1},  // e2a
    {64, 64, 3, 2},  // e2b
    {96, 32, 3, 1},  // d1a
    {32, 32, 3, 1},  // d1b
    {48, 16, 3, 1},  // d0a
    {16, 16, 3, 1},  // d0b
    {16, 16, 3, 1},  // out3
    {16, 4, 1, 1},   // out1
};
constexpr int pad16(int n) { return (n + 15) / 16 * 16; }
inline size_t frag_count(const Layer& L) {
  return (size_t)L.k * L.k * (pad16(L.cin) / 16) * (pad16(L.cout) / 16) * 64;
}
inline size_t packed_layer_bytes(const Layer& L) {
  return frag_count(L) * sizeof(bf16x4_t) + pad16(L.cout) * sizeof(float);
}
inline size_t param_offset(int i) {
  size_t o = 0;
  for (int j = 0; j < i; ++j) o += (size_t)kLayers[j].cout * kLayers[j].cin * kLayers[j].k * kLayers[j].k + kLayers[j].cout;
  return o;
}
inline size_t packed_offset(int i) {
  size_t o = 0;
  for (int j = 0; j < i; ++j) o += packed_layer_bytes(kLayers[j]);
  return o;
}
inline const bf16x4_t* layer_w(const void* packed, int i) {
  return reinterpret_cast<const bf16x4_t*>(static_cast<const char*>(packed) + packed_offset(i));
}
inline const float* layer_b(const void* packed, int i) {
  return reinterpret_cast<const float*>(static_cast<const char*>(packed) + packed_offset(i) +
                                        frag_count(kLayers[i]) * sizeof(bf16x4_t));
}

// Activation buffers in the workspace, in order: x0 (the prepared input,
// 16, full), e0 (16, full), t1 (32, full), e1 (32, half), t2 (64, half),
// e2 (64, quarter), t3 (32, half), d1 (32, half), t4 (16, full), t5 (16,
// full).
struct Grids {
  int H, W, Hh, Wh, Hq, Wq;
};
inline Grids grids(int H, int W) {
  Grids g{H, W, (H + 1) / 2, (W + 1) / 2, 0, 0};
  g.Hq = (g.Hh + 1) / 2;
  g.Wq = (g.Wh + 1) / 2;
  return g;
}
inline size_t align256(size_t n) { return (n + 255) / 256 * 256; }
constexpr int kActBufs = 10;
inline void act_layout(const Grids& g, size_t off[kActBufs + 1]) {
  const size_t full = (size_t)g.H * g.W * 2, half = (size_t)g.Hh * g.Wh * 2,
               quarter = (size_t)g.Hq * g.Wq * 2;
  const size_t sz[kActBufs] = {16 * full, 16 * full, 32 * full, 32 * half, 64 * half,
                               64 * quarter, 32 * half, 32 * half, 16 * full, 16 * full};
  off[0] = 0;
  for (int i = 0; i < kActBufs; ++i) off[i + 1] = off[i] + align256(sz[i]);
}

// Forward trace (flr_net_forward_trace): every layer's output activation,
// in the order of the header's layer table: x0 (the prepared input), in3,
// e0, e1a, e1, e2a, e2, d1a, d1, d0a, d0b, out3. The forward's own buffers
// (act_layout) come first; in3's and out3's outputs follow them.
constexpr int kTraceTensors = 12;
constexpr int kTraceChannels[kTraceTensors] = {16, 16, 16, 32, 32, 64, 64, 32, 32, 16, 16, 16};
constexpr int kTraceGrid[kTraceTensors] = {0, 0, 0, 0, 1, 1, 2, 1, 1, 0, 0, 0};
// trace index -> act_layout buffer (-1: the two stored after them)
constexpr int kTraceAct[kTraceTensors] = {0, -1, 1, 2, 3, 4, 5, 6, 7, 8, 9, -1};
inline void trace_layout(const Grids& g, size_t off[kTraceTensors + 1]) {
  size_t act[kActBufs + 1];
  act_layout(g, act);
  const size_t full16 = align256((size_t)g.H * g.W * 2 * 16);
  for (int i = 0; i < kTraceTensors; ++i)
    if (kTraceAct[i] >= 0) off[i] = act[kTraceAct[i]];
  off[1] = act[kActBufs];
  off[11] = act[kActBufs] + full16;
  off[kTraceTensors] = act[kActBufs] + 2 * full16;
}

bool valid_dims(int H, int W) {
  return H >= 1 && W >= 1 && H <= FLR_MAX_DIM && W <= FLR_MAX_DIM &&
         (int64_t)H * W <= ((int64_t)1 << 28);
}
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
  return a0 < b0 + nb && b0 < a0 + na;
}

template <int CIN, int COUT, int KS, int ST, int IN, int CUP, int FUSE, int COUT2>
hipError_t launch(const ConvArgs& a, hipStream_t s) {
  // (measured: the LDS tile is faster up to 48 input channels; at 96 its
  // 76 KB tile allows two workgroups per CU and the direct kernel wins)
  if constexpr (KS == 3 && ST == 1 && CIN <= 48) {
    auto k = conv_tile_kernel<CIN, COUT, IN, CUP, FUSE, COUT2>;
    const size_t lds = conv_tile_lds_bytes(CIN);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3((a.Wo + kTilePx - 1) / kTilePx, (a.Ho + kTileRows - 1) / kTileRows),
                       dim3(256), lds, s, a);
    return hipGetLastError();
  }
  constexpr int px_per_block = 4 * tiles_per_wave(CIN) * 16;
  hipLaunchKernelGGL((conv_kernel<CIN, COUT, KS, ST, IN, CUP, FUSE, COUT2>),
                     dim3((a.Wo + px_per_block - 1) / px_per_block, a.Ho), dim3(256), 0, s, a);
  return hipGetLastError();
}

// The forward pass into the activation buffers at the start of ws (the
// act_layout offsets), the sigmoid output planar FP32 into out. When set,
// mid_in3 and mid_out3 receive the activations of in3 and out3, which the
// fused kernels otherwise keep in registers (HWC BF16, 16 channels, full
// resolution).
flr_status run_forward(const Grids& g, const float* guides, const float* noisy, const void* packed,
                       float* out, char* ws, hipStream_t s, uint16_t* mid_in3 = nullptr,
                       uint16_t* mid_out3 = nullptr) {
  size_t off[kActBufs + 1];
  act_layout(g, off);
  auto buf = [&](int i) { return reinterpret_cast<uint16_t*>(ws + off[i]); };
  uint16_t *x0 = buf(0), *e0 = buf(1), *t1 = buf(2), *e1 = buf(3), *t2 = buf(4), *e2 = buf(5),
           *t3 = buf(6), *d1 = buf(7), *t4 = buf(8), *t5 = buf(9);
  auto args = [&](int layer, int Hi, int Wi, int Ho, int Wo) {
    ConvArgs a = {};
    a.w = layer_w(packed, layer);
    a.b = layer_b(packed, layer);
    a.Hi = Hi;
    a.Wi = Wi;
    a.Ho = Ho;
    a.Wo = Wo;
    return a;
  };
  hipError_t e;
  {  // input compression and layout
    const PrepArgs pa = {guides, noisy, x0, g.H, g.W};
    const size_t n = (size_t)g.H * g.W;
    hipLaunchKernelGGL(prep_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pa);
    if (hipGetLastError() != hipSuccess) return FLR_ERR_HIP;
  }
  {  // in3 + in1 -> e0
    ConvArgs a = args(0, g.H, g.W, g.H, g.W);
    a.in0 = x0;
    a.w2 = layer_w(packed, 1);
    a.b2 = layer_b(packed, 1);
    a.out = e0;
    a.mid = mid_in3;
    if ((e = launch<16, 16, 3, 1, IN_HWC, 0, FUSE_1X1_RELU, 16>(a, s)) != hipSuccess) return FLR_ERR_HIP;
  }
  {  // e1a
    ConvArgs a = args(2, g.H, g.W, g.H, g.W);
    a.in0 = e0;
    a.out = t1;
    if ((e = launch<16, 32, 3, 1, IN_HWC, 0, FUSE_NONE, 0>(a, s)) != hipSuccess) return FLR_ERR_HIP;
  }
  {  // e1b (stride 2)
    ConvArgs a = args(3, g.H, g.W, g.Hh, g.Wh);
    a.in0 = t1;
    a.out = e1;
    if ((e = launch<32, 32, 3, 2, IN_HWC, 0, FUSE_NONE, 0>(a, s)) != hipSuccess) return FLR_ERR_HIP;
  }
  {  // e2a
    ConvArgs a = args(4, g.Hh, g.Wh, g.Hh, g.Wh);
    a.in0 = e1;
    a.out = t2;
    if ((e = launch<32, 64, 3, 1, IN_HWC, 0, FUSE_NONE, 0>(a, s)) != hipSuccess) return FLR_ERR_HIP;
  }
  {  // e2b (stride 2)
    ConvArgs a = args(5, g.Hh, g.Wh, g.Hq, g.Wq);
    a.in0 = t2;
    a.out = e2;
    if ((e = launch<64, 64, 3, 2, IN_HWC, 0, FUSE_NONE, 0>(a, s)) != hipSuccess) return FLR_ERR_HIP;
  }
  {  // d1a: [up2(e2), e1]
    ConvArgs a = args(6, g.Hh, g.Wh, g.Hh, g.Wh);
    a.in0 = e2;
    a.Hl = g.Hq;
    a.Wl = g.Wq;
    a.in1 = e1;
    a.out = t3;
    if ((e = launch<96, 32, 3, 1, IN_UPCAT, 64, FUSE_NONE, 0>(a, s)) != hipSuccess) return FLR_ERR_HIP;
  }
  {  // d1b
    ConvArgs a = args(7, g.Hh, g.Wh, g.Hh, g.Wh);
    a.in0 = t3;
    a.out = d1;
    if ((e = launch<32, 32, 3, 1, IN_HWC, 0, FUSE_NONE, 0>(a, s)) != hipSuccess) return FLR_ERR_HIP;
  }
  {  // d0a: [up2(d1), e0]
    ConvArgs a = args(8, g.H, g.W, g.H, g.W);
    a.in0 = d1;
    a.Hl = g.Hh;
    a.Wl = g.Wh;
    a.in1 = e0;
    a.out = t4;
    if ((e = launch<48, 16, 3, 1, IN_UPCAT, 32, FUSE_NONE, 0>(a, s)) != hipSuccess) return FLR_ERR_HIP;
  }
  {  // d0b
    ConvArgs a = args(9, g.H, g.W, g.H, g.W);
    a.in0 = t4;
    a.out = t5;
    if ((e = launch<16, 16, 3, 1, IN_HWC, 0, FUSE_NONE, 0>(a, s)) != hipSuccess) return FLR_ERR_HIP;
  }
  {  // out3 + out1 (sigmoid) -> planar FP32
    ConvArgs a = args(10, g.H, g.W, g.H, g.W);
    a.in0 = t5;
    a.w2 = layer_w(packed, 11);
    a.b2 = layer_b(packed, 11);
    a.outf = out;
    a.mid = mid_out3;
    if ((e = launch<16, 16, 3, 1, IN_HWC, 0, FUSE_1X1_SIGMOID, FLR_NET_OUT>(a, s)) != hipSuccess)
      return FLR_ERR_HIP;
  }
  return FLR_OK;
}


}  // namespace flrnet

#include "flr_net_bwd.hpp"

namespace flrnet {

// Backward workspace: the forward's activation buffers (act_layout), then
// in3's and out3's activations (fused away in the forward), the sigmoid
// output, the BF16-rounded weights, the FP32 gradient tensors and the
// weight-gradient partials.
enum BwdBuf : int {
  B_A, B_T6, B_SIG, B_WR, B_DZ1, B_GT6, B_GT5, B_GT4, B_G48, B_GD1, B_GT3, B_G96, B_GE2, B_GT2,
  B_GE1, B_GT1, B_GE0, B_GA, B_PART, B_COUNT
};
// Output grid of each layer: 0 full, 1 half, 2 quarter.
constexpr int kOutGrid[12] = {0, 0, 0, 1, 1, 2, 1, 1, 0, 0, 0, 0};

inline size_t grid_px(const Grids& g, int which) {
  return which == 0 ? (size_t)g.H * g.W : which == 1 ? (size_t)g.Hh * g.Wh : (size_t)g.Hq * g.Wq;
}

inline void bwd_layout(const Grids& g, size_t off[B_COUNT + 1]) {
  size_t act[kActBufs + 1];
  act_layout(g, act);
  const size_t F = grid_px(g, 0), Hf = grid_px(g, 1), Q = grid_px(g, 2);
  size_t part = 0;
  for (int li = 0; li < 12; ++li) {
    const WgradPlan wp = wgrad_plan(kLayers[li], stored_cin_blocks(li), grid_px(g, kOutGrid[li]));
    const size_t S = (size_t)wp.ne * kWgAcc + kLayers[li].cout;
    const size_t n = ((size_t)wp.nchunk + (wp.nchunk + kChunkGroup - 1) / kChunkGroup) * S;
    if (n > part) part = n;
  }
  const size_t sz[B_COUNT] = {16 * F * 2,  16 * F * 2,  4 * F * 4,   param_offset(12) * 4,
                              4 * F * 4,   16 * F * 4,  16 * F * 4,  16 * F * 4,
                              48 * F * 4,  32 * Hf * 4, 32 * Hf * 4, 96 * Hf * 4,
                              64 * Q * 4,  64 * Hf * 4, 32 * Hf * 4, 32 * F * 4,
                              16 * F * 4,  16 * F * 4,  part * 4};
  off[0] = act[kActBufs];
  for (int i = 0; i < B_COUNT; ++i) off[i + 1] = off[i] + align256(sz[i]);
}

// Weight and bias gradients of layer li: chunked partials, then the
// fixed-order sum into grad (+= when accumulate).
hipError_t layer_wgrad(int li, const Grids& g, const float* gout, const uint16_t* act,
                       const BwdSrc& src, int Hi, int Wi, float* part, float* grad, int accumulate,
                       hipStream_t s) {
  const Layer& L = kLayers[li];
  const int ncb = stored_cin_blocks(li);
  const int og = kOutGrid[li];
  const int Ho = og == 0 ? g.H : og == 1 ? g.Hh : g.Hq, Wo = og == 0 ? g.W : og == 1 ? g.Wh : g.Wq;
  const WgradPlan wp = wgrad_plan(L, ncb, (size_t)Ho * Wo);
  WgradArgs a = {};
  a.g = gout;
  a.act = act;
  a.src = src;
  a.Hi = Hi;
  a.Wi = Wi;
  a.Ho = Ho;
  a.Wo = Wo;
  a.cout = L.cout;
  a.ncb = ncb;
  a.k = L.k;
  a.stride = L.stride;
  a.ne = wp.ne;
  a.chunk_px = wp.chunk_px;
  a.part = part;
  if (L.k == 3)
    hipLaunchKernelGGL(wgrad_kernel<3>, dim3(wp.nchunk, wp.wg_y), dim3(256), wgrad_lds_bytes(), s,
                       a);
  else
    hipLaunchKernelGGL(wgrad_kernel<1>, dim3(wp.nchunk, wp.wg_y), dim3(256), wgrad_lds_bytes(), s,
                       a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // two-level fixed-order sum over the chunks: groups of kChunkGroup, then the groups
  const int S = wp.ne * kWgAcc + L.cout;
  const int ng = (wp.nchunk + kChunkGroup - 1) / kChunkGroup;
  float* groups = part + (size_t)wp.nchunk * S;
  const ChunkSumArgs c = {part, groups, S, wp.nchunk};
  const size_t nc = (size_t)ng * S;
  hipLaunchKernelGGL(chunk_sum_kernel, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, c);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const WreduceArgs r = {groups, ng, wp.ne, ncb, L.cin, L.cout, L.k, grad + param_offset(li),
                         accumulate};
  hipLaunchKernelGGL(wreduce_kernel, dim3((S + 255) / 256), dim3(256), 0, s, r);
  return hipGetLastError();
}

// Pixel count from which the data gradients take 16 input channels per
// thread: FLR_DGRAD_WIDE_PX from the environment when it holds a number (a
// tuning knob; the gradients are bit-identical either way, the sum order per
// channel being the same), else kDgWidePx.
static size_t dgrad_wide_px() {
  const char* e = getenv("FLR_DGRAD_WIDE_PX");
  if (e && *e) {
    char* end = nullptr;
    const long long v = strtoll(e, &end, 10);
    if (end && *end == 0 && v >= 0) return (size_t)v;
  }
  return kDgWidePx;
}

// Gradient of layer li's input (channels 0..cin-1, HWC FP32 into dx), plus
// an optional addend tensor's channels.
hipError_t layer_dgrad(int li, const Grids& g, const float* gout, const uint16_t* act,
                       const float* wr, int Hi, int Wi, float* dx, const float* add, int add_cs,
                       int add_off, hipStream_t s) {
  const Layer& L = kLayers[li];
  const size_t n = (size_t)Hi * Wi;
  const int cpt = n >= dgrad_wide_px() ? 16 : 8;
  if (L.cin % cpt) return hipErrorInvalidValue;  // whole channel groups per thread
  const int og = kOutGrid[li];
  DgradArgs a = {};
  a.g = gout;
  a.act = act;
  a.w = wr + param_offset(li);
  a.cin = L.cin;
  a.cout = L.cout;
  a.k = L.k;
  a.stride = L.stride;
  a.Hi = Hi;
  a.Wi = Wi;
  a.Ho = og == 0 ? g.H : og == 1 ? g.Hh : g.Hq;
  a.Wo = og == 0 ? g.W : og == 1 ? g.Wh : g.Wq;
  a.dx = dx;
  a.add = add;
  a.add_cs = add_cs;
  a.add_off = add_off;
  if (cpt == 16)
    hipLaunchKernelGGL(dgrad_kernel<16>, dim3((unsigned)((n + 255) / 256), L.cin / 16), dim3(256),
                       dgrad_lds_bytes(L, 16), s, a);
  else
    hipLaunchKernelGGL(dgrad_kernel<8>, dim3((unsigned)((n + 255) / 256), L.cin / 8), dim3(256),
                       dgrad_lds_bytes(L, 8), s, a);
  return hipGetLastError();
}

hipError_t up2_bwd(const float* fine, int H, int W, int cs, float* low, int Hl, int Wl, int nc,
                   hipStream_t s) {
  const size_t n = (size_t)Hl * Wl * nc;
  const Up2BwdArgs a = {fine, H, W, cs, low, Hl, Wl, nc};
  hipLaunchKernelGGL(up2_bwd_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

flr_status run_backward(const Grids& g, const float* guides, const float* noisy,
                        const float* params, const void* packed, const float* dout, float* grad,
                        int accumulate, char* ws, hipStream_t s) {
  size_t act[kActBufs + 1], off[B_COUNT + 1];
  act_layout(g, act);
  bwd_layout(g, off);
  auto abuf = [&](int i) { return reinterpret_cast<uint16_t*>(ws + act[i]); };
  auto fbuf = [&](int i) { return reinterpret_cast<float*>(ws + off[i]); };
  uint16_t *x0 = abuf(0), *e0 = abuf(1), *t1 = abuf(2), *e1 = abuf(3), *t2 = abuf(4),
           *e2 = abuf(5), *t3 = abuf(6), *d1 = abuf(7), *t4 = abuf(8), *t5 = abuf(9);
  uint16_t* a16 = reinterpret_cast<uint16_t*>(ws + off[B_A]);
  uint16_t* t6 = reinterpret_cast<uint16_t*>(ws + off[B_T6]);
  float *sig = fbuf(B_SIG), *wr = fbuf(B_WR), *part = fbuf(B_PART);
  const int F = (int)grid_px(g, 0);
  const int np = (int)param_offset(12);

  const RoundArgs ra = {params, wr, np};
  hipLaunchKernelGGL(round_params_kernel, dim3((np + 255) / 256), dim3(256), 0, s, ra);
  if (hipGetLastError() != hipSuccess) return FLR_ERR_HIP;
  // the forward, also storing in3's and out3's activations
  flr_status st = run_forward(g, guides, noisy, packed, sig, ws, s, a16, t6);
  if (st != FLR_OK) return st;
  const SigmoidBwdArgs sa = {dout, sig, fbuf(B_DZ1), F, FLR_NET_OUT};
  hipLaunchKernelGGL(sigmoid_bwd_kernel, dim3((F + 255) / 256), dim3(256), 0, s, sa);
  if (hipGetLastError() != hipSuccess) return FLR_ERR_HIP;

  auto plain = [](const uint16_t* in, int cs) { return BwdSrc{in, nullptr, cs, cs, 0, 0}; };
  const BwdSrc cat48 = {d1, e0, 32, 32, 16, g.Wh};
  const BwdSrc cat96 = {e2, e1, 64, 64, 32, g.Wq};
  bool ok = true;
  auto W = [&](int li, const float* go, const uint16_t* ac, const BwdSrc& src, int Hi, int Wi) {
    ok = ok && layer_wgrad(li, g, go, ac, src, Hi, Wi, part, grad, accumulate, s) == hipSuccess;
  };
  auto D = [&](int li, const float* go, const uint16_t* ac, int Hi, int Wi, float* dx,
               const float* add = nullptr, int add_cs = 0, int add_off = 0) {
    ok = ok && layer_dgrad(li, g, go, ac, wr, Hi, Wi, dx, add, add_cs, add_off, s) == hipSuccess;
  };
  // out1 (sigmoid head, no mask) and the layers back to in3, as in the forward reversed
  W(11, fbuf(B_DZ1), nullptr, plain(t6, 16), g.H, g.W);
  D(11, fbuf(B_DZ1), nullptr, g.H, g.W, fbuf(B_GT6));
  W(10, fbuf(B_GT6), t6, plain(t5, 16), g.H, g.W);
  D(10, fbuf(B_GT6), t6, g.H, g.W, fbuf(B_GT5));
  W(9, fbuf(B_GT5), t5, plain(t4, 16), g.H, g.W);
  D(9, fbuf(B_GT5), t5, g.H, g.W, fbuf(B_GT4));
  W(8, fbuf(B_GT4), t4, cat48, g.H, g.W);
  D(8, fbuf(B_GT4), t4, g.H, g.W, fbuf(B_G48));
  ok = ok && up2_bwd(fbuf(B_G48), g.H, g.W, 48, fbuf(B_GD1), g.Hh, g.Wh, 32, s) == hipSuccess;
  W(7, fbuf(B_GD1), d1, plain(t3, 32), g.Hh, g.Wh);
  D(7, fbuf(B_GD1), d1, g.Hh, g.Wh, fbuf(B_GT3));
  W(6, fbuf(B_GT3), t3, cat96, g.Hh, g.Wh);
  D(6, fbuf(B_GT3), t3, g.Hh, g.Wh, fbuf(B_G96));
  ok = ok && up2_bwd(fbuf(B_G96), g.Hh, g.Wh, 96, fbuf(B_GE2), g.Hq, g.Wq, 64, s) == hipSuccess;
  W(5, fbuf(B_GE2), e2, plain(t2, 64), g.Hh, g.Wh);
  D(5, fbuf(B_GE2), e2, g.Hh, g.Wh, fbuf(B_GT2));
  W(4, fbuf(B_GT2), t2, plain(e1, 32), g.Hh, g.Wh);
  D(4, fbuf(B_GT2), t2, g.Hh, g.Wh, fbuf(B_GE1), fbuf(B_G96), 96, 64);
  W(3, fbuf(B_GE1), e1, plain(t1, 32), g.H, g.W);
  D(3, fbuf(B_GE1), e1, g.H, g.W, fbuf(B_GT1));
  W(2, fbuf(B_GT1), t1, plain(e0, 16), g.H, g.W);
  D(2, fbuf(B_GT1), t1, g.H, g.W, fbuf(B_GE0), fbuf(B_G48), 48, 32);
  W(1, fbuf(B_GE0), e0, plain(a16, 16), g.H, g.W);
  D(1, fbuf(B_GE0), e0, g.H, g.W, fbuf(B_GA));
  W(0, fbuf(B_GA), a16, plain(x0, 16), g.H, g.W);
  return ok ? FLR_OK : FLR_ERR_HIP;
}
}  // namespace flrnet

using namespace flrnet;

extern "C" {

size_t flr_net_num_params(void) { return param_offset(12); }

size_t flr_net_packed_bytes(void) { return packed_offset(12); }

flr_status flr_net_pack(const float* params, void* packed, void* stream) {
  if (!params || !packed) return FLR_ERR_NULL;
  if (!aligned16(params) || !aligned16(packed)) return FLR_ERR_ALIGN;
  if (overlaps(params, flr_net_num_params() * sizeof(float), packed, flr_net_packed_bytes()))
    return FLR_ERR_ALIAS;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (int i = 0; i < 12; ++i) {
    const Layer& L = kLayers[i];
    const float* w = params + param_offset(i);
    const float* b = w + (size_t)L.cout * L.cin * L.k * L.k;
    const int n = (int)frag_count(L);
    const PackArgs pa = {w, b, L.cin, L.cout, L.k, pad16(L.cin) / 16, pad16(L.cout) / 16,
                         const_cast<bf16x4_t*>(layer_w(packed, i)),
                         const_cast<float*>(layer_b(packed, i))};
    hipLaunchKernelGGL(pack_kernel, dim3((n + 255) / 256), dim3(256), 0, s, pa);
    if (hipGetLastError() != hipSuccess) return FLR_ERR_HIP;
  }
  return FLR_OK;
}

size_t flr_net_workspace_bytes(int32_t height, int32_t width) {
  if (!valid_dims(height, width)) return 0;
  size_t off[kActBufs + 1];
  act_layout(grids(height, width), off);
  return off[kActBufs];
}

flr_status flr_net_forward(int32_t height, int32_t width, const float* guides, const float* noisy,
                           const void* packed, float* out, void* workspace, size_t workspace_bytes,
                           void* stream) {
  if (!valid_dims(height, width)) return FLR_ERR_SHAPE;
  if (!guides || !noisy || !packed || !out) return FLR_ERR_NULL;
  if (!aligned16(guides) || !aligned16(noisy) || !aligned16(packed) || !aligned16(out))
    return FLR_ERR_ALIGN;
  const size_t need = flr_net_workspace_bytes(height, width);
  if (!workspace || workspace_bytes < need) return FLR_ERR_WORKSPACE;
  if (!aligned16(workspace)) return FLR_ERR_ALIGN;
  const size_t pb = (size_t)height * width * sizeof(float);
  const size_t gb = FLR_NET_IN_GUIDES * pb, nb = FLR_NET_IN_NOISY * pb, ob = FLR_NET_OUT * pb;
  const size_t kb = flr_net_packed_bytes();
  if (overlaps(out, ob, guides, gb) || overlaps(out, ob, noisy, nb) || overlaps(out, ob, packed, kb) ||
      overlaps(workspace, need, guides, gb) || overlaps(workspace, need, noisy, nb) ||
      overlaps(workspace, need, packed, kb) || overlaps(workspace, need, out, ob))
    return FLR_ERR_ALIAS;
  return run_forward(grids(height, width), guides, noisy, packed, out,
                     static_cast<char*>(workspace), reinterpret_cast<hipStream_t>(stream));
}

size_t flr_net_trace_bytes(int32_t height, int32_t width) {
  if (!valid_dims(height, width)) return 0;
  size_t off[kTraceTensors + 1];
  trace_layout(grids(height, width), off);
  return off[kTraceTensors];
}

flr_status flr_net_trace_tensor(int32_t height, int32_t width, int32_t index, size_t* offset,
                                int32_t* channels, int32_t* tensor_height, int32_t* tensor_width) {
  if (!valid_dims(height, width)) return FLR_ERR_SHAPE;
  if (!offset || !channels || !tensor_height || !tensor_width) return FLR_ERR_NULL;
  if (index < 0 || index >= kTraceTensors) return FLR_ERR_MODE;
  const Grids g = grids(height, width);
  size_t off[kTraceTensors + 1];
  trace_layout(g, off);
  const int which = kTraceGrid[index];
  *offset = off[index];
  *channels = kTraceChannels[index];
  *tensor_height = which == 0 ? g.H : which == 1 ? g.Hh : g.Hq;
  *tensor_width = which == 0 ? g.W : which == 1 ? g.Wh : g.Wq;
  return FLR_OK;
}

flr_status flr_net_forward_trace(int32_t height, int32_t width, const float* guides,
                                 const float* noisy, const void* packed, float* out, void* trace,
                                 size_t trace_bytes, void* stream) {
  if (!valid_dims(height, width)) return FLR_ERR_SHAPE;
  if (!guides || !noisy || !packed || !out) return FLR_ERR_NULL;
  if (!aligned16(guides) || !aligned16(noisy) || !aligned16(packed) || !aligned16(out))
    return FLR_ERR_ALIGN;
  const size_t need = flr_net_trace_bytes(height, width);
  if (!trace || trace_bytes < need) return FLR_ERR_WORKSPACE;
  if (!aligned16(trace)) return FLR_ERR_ALIGN;
  const size_t pb = (size_t)height * width * sizeof(float);
  const size_t gb = FLR_NET_IN_GUIDES * pb, nb = FLR_NET_IN_NOISY * pb, ob = FLR_NET_OUT * pb;
  const size_t kb = flr_net_packed_bytes();
  if (overlaps(out, ob, guides, gb) || overlaps(out, ob, noisy, nb) || overlaps(out, ob, packed, kb) ||
      overlaps(trace, need, guides, gb) || overlaps(trace, need, noisy, nb) ||
      overlaps(trace, need, packed, kb) || overlaps(trace, need, out, ob))
    return FLR_ERR_ALIAS;
  const Grids g = grids(height, width);
  size_t off[kTraceTensors + 1];
  trace_layout(g, off);
  char* t = static_cast<char*>(trace);
  return run_forward(g, guides, noisy, packed, out, t, reinterpret_cast<hipStream_t>(stream),
                     reinterpret_cast<uint16_t*>(t + off[1]),
                     reinterpret_cast<uint16_t*>(t + off[11]));
}

size_t flr_net_backward_workspace_bytes(int32_t height, int32_t width) {
  if (!valid_dims(height, width)) return 0;
  size_t off[B_COUNT + 1];
  bwd_layout(grids(height, width), off);
  return off[B_COUNT];
}

flr_status flr_net_backward(int32_t height, int32_t width, const float* guides, const float* noisy,
                            const float* params, const void* packed, const float* grad_out,
                            float* grad_params, int32_t accumulate, void* workspace,
                            size_t workspace_bytes, void* stream) {
  if (!valid_dims(height, width)) return FLR_ERR_SHAPE;
  if (!guides || !noisy || !params || !packed || !grad_out || !grad_params) return FLR_ERR_NULL;
  if (!aligned16(guides) || !aligned16(noisy) || !aligned16(params) || !aligned16(packed) ||
      !aligned16(grad_out) || !aligned16(grad_params))
    return FLR_ERR_ALIGN;
  if (accumulate != 0 && accumulate != 1) return FLR_ERR_MODE;
  const size_t need = flr_net_backward_workspace_bytes(height, width);
  if (!workspace || workspace_bytes < need) return FLR_ERR_WORKSPACE;
  if (!aligned16(workspace)) return FLR_ERR_ALIGN;
  const size_t pb = (size_t)height * width * sizeof(float);
  const size_t gb = FLR_NET_IN_GUIDES * pb, nb = FLR_NET_IN_NOISY * pb, ob = FLR_NET_OUT * pb;
  const size_t kb = flr_net_packed_bytes(), wb = flr_net_num_params() * sizeof(float);
  const void* ins[5] = {guides, noisy, params, packed, grad_out};
  const size_t inb[5] = {gb, nb, wb, kb, ob};
  for (int i = 0; i < 5; ++i)
    if (overlaps(workspace, need, ins[i], inb[i]) || overlaps(grad_params, wb, ins[i], inb[i]))
      return FLR_ERR_ALIAS;
  if (overlaps(workspace, need, grad_params, wb)) return FLR_ERR_ALIAS;
  return run_backward(grids(height, width), guides, noisy, params, packed, grad_out, grad_params,
                      accumulate, static_cast<char*>(workspace),
                      reinterpret_cast<hipStream_t>(stream));
}

size_t flr_flnr_workspace_bytes(const flr_params* p) {
  if (!p || flr_validate_params(p) != FLR_OK) return 0;
  if (p->num_guides != FLR_NET_IN_GUIDES + FLR_NET_OUT || p->num_channels != FLR_NET_IN_NOISY)
    return 0;
  return align256(flr_denoise_workspace_bytes(p)) + flr_net_workspace_bytes(p->height, p->width);
}

flr_status flr_flnr_denoise(const flr_params* p, float* guides12, const float* noisy,
                            const void* packed, float* out, void* workspace,
                            size_t workspace_bytes, void* stream) {
  flr_status st = flr_validate_params(p);
  if (st != FLR_OK) return st;
  if (p->num_guides != FLR_NET_IN_GUIDES + FLR_NET_OUT || p->num_channels != FLR_NET_IN_NOISY)
    return FLR_ERR_CHANNELS;
  if (p->flags & FLR_FLAG_RAW_MOMENTS) return FLR_ERR_MODE;
  if (!guides12 || !noisy || !packed || !out) return FLR_ERR_NULL;
  const size_t need = flr_flnr_workspace_bytes(p);
  if (!workspace || workspace_bytes < need) return FLR_ERR_WORKSPACE;
  const size_t pl = (size_t)p->height * p->width;
  const size_t fw = align256(flr_denoise_workspace_bytes(p));
  char* ws = static_cast<char*>(workspace);
  st = flr_net_forward(p->height, p->width, guides12, noisy, packed,
                       guides12 + FLR_NET_IN_GUIDES * pl, ws + fw, need - fw, stream);
  if (st != FLR_OK) return st;
  return flr_denoise(p, guides12, noisy, out, fw ? ws : nullptr, fw, stream);
}

}  // extern "C"
