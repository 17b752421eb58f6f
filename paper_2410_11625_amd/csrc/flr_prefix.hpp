// Horizontal window sums by segmented prefix sums (DPP lane moves and LDS),
// shared by the walkers, the averaging kernel and the box passes.
#pragma once

#include <hip/hip_runtime.h>

#include "flr_launch.hpp"

namespace flr {

// Horizontal window sums by segmented prefix sums. Lane l holds the value x_l
// of its column. An inclusive prefix over aligned segments of L lanes (L = 16,
// one DPP row, when 2r <= 16; else L = 64, the wavefront) is formed in
// registers with DPP lane moves, log2(L) add steps, and staged through LDS
// once. A window [j, j + 2r] with 2r <= L touches at most two segments, so its
// sum is P[j + 2r] - P[j - 1] + (P[end of j's segment] if it crosses), with
// P[j - 1] dropped when j starts a segment: three independent LDS reads in
// place of a serial slide. Segments never cross a wavefront.

// DPP control codes (GFX9 encoding): row_shr:k, row_bcast:15, row_bcast:31.
constexpr int kDppRowShr = 0x110;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;
constexpr int kDppWaveShr1 = 0x138;

// x of the DPP source lane (0 where the source is outside the row, or the
// lane's row is masked off), 64-bit values as two 32-bit moves.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, ROW_MASK, 0xf, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_move(float x) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, true));
}

// Inclusive prefix of x over its 16-lane row, or over the wavefront (WIDE).
// Every lane of the wavefront must take part.
template <bool WIDE, typename E>
__device__ __forceinline__ E seg_prefix(E x) {
  x += dpp_move<kDppRowShr + 1, 0xf>(x);
  x += dpp_move<kDppRowShr + 2, 0xf>(x);
  x += dpp_move<kDppRowShr + 4, 0xf>(x);
  x += dpp_move<kDppRowShr + 8, 0xf>(x);
  if (WIDE) {
    x += dpp_move<kDppRowBcast15, 0xa>(x);  // row totals 0 -> 1, 2 -> 3
    x += dpp_move<kDppRowBcast31, 0xc>(x);  // rows 0..1 total -> 2, 3
  }
  return x;
}

// Value of the lane to the left within the prefix segment (0 at its start).
template <bool WIDE, typename E>
__device__ __forceinline__ E seg_left(E x) {
  return WIDE ? dpp_move<kDppWaveShr1, 0xf>(x) : dpp_move<kDppRowShr + 1, 0xf>(x);
}

// seg_prefix of N values at once, step by step across the values, so that
// independent moves and adds overlap each other's latency.
template <int CTRL, int ROW_MASK, int N, typename E>
__device__ __forceinline__ void seg_step(E (&x)[N]) {
  E t[N];
#pragma unroll
  for (int i = 0; i < N; ++i) t[i] = dpp_move<CTRL, ROW_MASK>(x[i]);
  // keep the N moves ahead of their adds (independent work between a
  // move and the add that reads it)
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] += t[i];
}
template <bool WIDE, int N, typename E>
__device__ __forceinline__ void seg_prefix_n(E (&x)[N]) {
  seg_step<kDppRowShr + 1, 0xf>(x);
  seg_step<kDppRowShr + 2, 0xf>(x);
  seg_step<kDppRowShr + 4, 0xf>(x);
  seg_step<kDppRowShr + 8, 0xf>(x);
  if (WIDE) {
    seg_step<kDppRowBcast15, 0xa>(x);  // row totals 0 -> 1, 2 -> 3
    seg_step<kDppRowBcast31, 0xc>(x);  // rows 0..1 total -> 2, 3
  }
}

// Prefix segments of 16 lanes serve windows up to 2r + 1 = 17 columns wide.
__host__ __device__ constexpr bool wide_segments(int r) { return r > 8; }

// LDS columns whose prefixes give the sum of window [j, j + 2r]:
// P[ib] - P[ia] + P[it]. Terms that do not apply point at the row's pad
// column kThreads, which holds zero.
struct HWin {
  int ib, ia, it;
};
template <bool WIDE>
__device__ __forceinline__ HWin hwin(int j, int r) {
  constexpr int lm = WIDE ? 63 : 15;
  HWin h;
  h.ib = min(j + 2 * r, kThreads - 1);
  h.ia = (j & lm) != 0 ? j - 1 : kThreads;
  h.it = (h.ib & ~lm) != (j & ~lm) ? (j | lm) : kThreads;
  return h;
}
template <typename E>
__device__ __forceinline__ E hwin_sum(const E* row, const HWin& h) {
  return (row[h.ib] - row[h.ia]) + row[h.it];
}

// x itself, moved through DPP with the identity quad permutation. The
// compiler cannot prove the result loop-invariant, so LDS addresses formed
// from it inside a loop are formed there (a few adds, immediate offsets)
// instead of being hoisted out as hundreds of precomputed addresses.
__device__ __forceinline__ int lane_opaque(int x) {
  return __builtin_amdgcn_update_dpp(0, x, 0xE4, 0xf, 0xf, false);
}
__device__ __forceinline__ HWin hwin_opaque(const HWin& h) {
  HWin o;
  o.ib = lane_opaque(h.ib);
  o.ia = lane_opaque(h.ia);
  o.it = lane_opaque(h.it);
  return o;
}

}  // namespace flr
