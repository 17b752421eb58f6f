// Launch geometry and the interface between the host dispatcher and the
// per-guide-count kernel instantiations. Host and device code share it.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace flr {

// One workgroup = one column strip of kThreads input columns walking down a
// segment of rows. Four 64-wide wavefronts.
constexpr int kThreads = 256;
// MI355X compute units; the automatic segment choice aims for whole waves of
// workgroups over this many CUs (the walker kernels run one workgroup per CU).
constexpr int kCUs = 256;
// Numeric types. Products of the FP32 inputs are summed in sum_t; central
// moments, intercepts, the coefficient average and the reconstruction run in
// solve_t; the centred, regularised system is factorised and solved in
// chol_t (it is well conditioned once centred in solve_t). (With packed FP32 unused, an FP64 FMA
// issues at the same rate as an FP32 one on CDNA4; FP64 costs registers and
// LDS bytes, not ALU slots.)
#ifndef FLR_SUM_T
#define FLR_SUM_T double
#endif
#ifndef FLR_SOLVE_T
#define FLR_SOLVE_T double
#endif
// Element type of the fused kernel's coefficient ring (coefficients relative
// to the workgroup anchor).
#ifndef FLR_RING_T
#define FLR_RING_T float
#endif
// Factorisation and triangular solves of the per-pixel system. FP64: with
// the regulariser at 1e-3 of unit-scale guides, windows of near-constant
// guides make the centred system's condition number reach 1e4 and more, and
// an FP32 factorisation then errs by up to 2e-4 relative in the output
// (measured on 40 x 270 frames of the RGB workload); in FP64 it is below 2e-5.
#ifndef FLR_CHOL_T
#define FLR_CHOL_T double
#endif
typedef FLR_CHOL_T chol_t;
typedef FLR_SUM_T sum_t;
typedef FLR_SOLVE_T solve_t;
typedef FLR_RING_T ring_t;
// Running vertical sums of the ring values in the fused kernel.
#ifndef FLR_AVG_T
#define FLR_AVG_T double
#endif
typedef FLR_AVG_T avg_t;
// LDS row stride in elements: kThreads + 1 keeps lanes that read
// consecutive channel rows of one column on distinct banks.
constexpr int kLdsStride = kThreads + 1;
// LDS per workgroup (gfx950: 160 KiB).
constexpr int kLdsBytes = 163840;
// Channel rows of element size `elem` that fit twice (source and
// destination of the horizontal pass) in LDS.
__host__ __device__ constexpr int max_lds_rows(int elem) {
  return kLdsBytes / (2 * kLdsStride * elem);
}
__host__ __device__ constexpr int group_count(int rows, int elem) {
  return (rows + max_lds_rows(elem) - 1) / max_lds_rows(elem);
}
__host__ __device__ constexpr int group_size(int rows, int elem) {
  return (rows + group_count(rows, elem) - 1) / group_count(rows, elem);
}

enum Kind : int {
  K_MOMENTS = 0,      // window moments -> moment planes
  K_SOLVE = 1,        // moment planes -> coefficient planes
  K_APPLY_POINT = 2,  // coefficient planes + guides -> output (no averaging)
  K_APPLY_AVG = 3,    // coefficient planes -> window average -> output
  K_FUSED0 = 4,       // moments -> solve -> apply, no averaging, one kernel
  K_FUSED1 = 5,       // moments -> solve -> average -> apply, one kernel
  K_COEFFS = 6,       // moments -> solve -> coefficient planes, one kernel
  K_MOMENTS_A = 7,    // K_MOMENTS over the first slice of the product channels
  K_MOMENTS_B = 8,    // K_MOMENTS over the rest (split walks)
  // adjoint (flr_denoise_backward)
  K_ADJ_COEF = 9,     // coefficients from FP64 moment sums + the averaging fields
  K_ADJ_SOLVE = 10,   // per-pixel solve adjoint -> fields whose window sums give dL/dg, dL/dy
  K_ADJ_GATHER = 11,  // window sums of those fields contracted with g and y
  // the downsampled-moment variant (flr_denoise_lowres)
  K_LR_BLOCK = 12,    // block sums of the anchored products -> low-resolution planes
  K_LR_SOLVE = 13,    // Gaussian pass along columns + solve per low-resolution pixel
  K_LR_APPLY = 14,    // bilinear model interpolation + reconstruction
  // batched serving
  K_COEFFS_BATCH = 15,     // K_COEFFS over the tiles of several frames
  K_APPLY_AVG_BATCH = 16,  // K_APPLY_AVG over the tiles of several frames
  K_UP_APPLY_BATCH = 17,   // bilinear upsampling of coefficient planes + reconstruction
  K_BATCH_PERSISTENT = 18, // every stage of a batch in one launch over a work queue
  K_SPLIT_COEFFS = 19,     // split walks: the walk over the second slice, with the first
                           // slice's moment planes read back -> solve -> coefficient planes
};

// One persistent launch for a batch (flr_batch_run): workgroups take items
// from a queue counter in order; an item is one workgroup's tile of one
// stage of one frame. Stages, in queue order: the coefficient walk of the
// plain frames; per joint frame the FP64 window sums of its products, the
// per-pixel solve and the window mean of the models; the averaging and
// reconstruction of the plain frames; the upsampling of the joint frames.
// An item only waits on items earlier in the queue (taken by workgroups
// that are running), through counters that finished items increment.
enum BatchItemKind : int {
  BI_WALK = 0, BI_JBOX = 1, BI_JSOLVE = 2, BI_JMEAN = 3, BI_AVG = 4, BI_UP = 5
};
struct BatchStage {
  int kind;      // BatchItemKind
  int arg;       // index into the launch-argument table (largs) or, box passes, bargs
  int first;     // first queue item of the stage
  int count;     // its items
  int nx;        // box passes: workgroups per plane
  int wait;      // counter its items wait on (-1: none); BI_AVG: the frame's
                 // first walk-segment counter
  int need;      // the value that counter must reach (BI_AVG: strips per walk segment)
  int done;      // counter a finished item increments (-1: none); BI_WALK: the
                 // frame's first walk-segment counter (one per segment)
  int seg_rows;  // BI_WALK, BI_AVG: rows per walk segment of the frame
  int nseg;      // BI_AVG: walk segments of the frame
};
// Arguments of one box pass (flr_box.hpp).
struct AdjBoxArgs {
  const float* srcf;   // BOX_MEAN32: FP32 planes, averaged into dstf
  float* dstf;
  const double* src;   // FP64 planes, or NULL for the product channels below
  const float* guides; // product channels: guides [Q][H][W]
  const float* noisy;  // product channels: noisy [C][H][W]
  const float* gout;   // BOX_AVGFIELDS: dL/d(output) [C][H][W]
  double* dst;
  int64_t plane;  // elements per plane
  int H, W, r, seg_rows, tiles_x;
  int Q, C;
  int count_first;  // BOX_PRODUCTS: plane 0 is the window pixel count, channels follow
  int ring;         // 1: the leaving rows come from an LDS ring of 2r + 1 rows
};

// LDS bytes of a box pass: two FP64 prefix rows of kThreads + 1, and with
// the ring 2r + 1 FP64 rows of kThreads.
inline size_t box_lds_bytes(int r, bool ring) {
  return (size_t)(2 * (kThreads + 1) + (ring ? (2 * r + 1) * kThreads : 0)) * sizeof(double);
}
// Largest LDS of a standalone box launch with the ring (so that several
// workgroups share a CU); larger radii load the leaving row again.
constexpr size_t kBoxLdsMax = 64 * 1024;

// Rows per workgroup segment of a box pass, and its tiling: sets plane,
// seg_rows, tiles_x; returns the workgroups per plane. Segments of up to
// kBoxSegRows rows (each repeats 2r warm-up rows), halved while the
// `planes` planes of the pass would give fewer than kBoxMinGroups
// workgroups.
constexpr int kBoxSegRows = 128;
constexpr int kBoxMinGroups = 2048;
inline int box_plan(AdjBoxArgs& a, int planes = 1) {
  a.plane = (int64_t)a.H * a.W;
  a.tiles_x = (a.W + (kThreads - 2 * a.r) - 1) / (kThreads - 2 * a.r);
  int seg = kBoxSegRows;
  while (seg > 16 && (int64_t)a.tiles_x * ((a.H + seg - 1) / seg) * planes < kBoxMinGroups)
    seg /= 2;
  a.seg_rows = seg < a.H ? seg : a.H;
  return a.tiles_x * ((a.H + a.seg_rows - 1) / a.seg_rows);
}

struct BatchPlanDev {
  const BatchStage* stages;
  int nstages, nitems, ncounters, pad;
  const struct LaunchArgs* largs;
  const AdjBoxArgs* bargs;
  int* ctl;       // [0] queue head, [1] workgroups finished, [2] waits given up (kept)
  int* counters;  // [ncounters]
};
// Longest wait of an item before it gives up and flags the run as failed
// (iterations of a short sleep; far beyond any item's duration).
constexpr int kBatchSpinLimit = 1 << 24;

// Longest Gaussian of the downsampled-moment variant (taps -R..R).
constexpr int kMaxLowresRadius = 8;

struct LaunchArgs {
  const float* guides;   // [Q][H][W]
  const float* noisy;    // [C][H][W]
  const float* planes;   // K_SOLVE: moments; K_APPLY_*: coefficients
  float* out;            // moments / coefficients / output image
  void* ring;            // K_FUSED1 workspace (ring_t elements)
  int H, W, r;
  int seg_rows, tiles_x, n_seg;
  int hchunk_m, hchunk_a;  // horizontal-pass chunk lengths (moments, averaging)
  float eps, eps_mul;
  const float* eps_dev;  // when set: (eps, eps_mul) read from device memory instead
  int reg_mode;
  int raw;
  // K_COEFFS / K_SPLIT_COEFFS / K_APPLY_AVG (and their batched forms): the
  // coefficient image carries each intercept as an FP32 pair, hi in plane c
  // and lo in plane (Q + 1) C + c, formed in FP64 from the slopes as stored
  // (FP32), so that the model's value at the window mean is kept to FP64
  // accuracy where a fit's intercept and slope terms cancel
  int coef_lo;
  // adjoint kernels only
  const float* gout;     // dL/d(output) [C][H][W]
  const float* coeffs;   // unaveraged coefficient planes (b | a)
  const double* sums;    // FP64 window sums of the anchored input products
  const double* fin;     // FP64 field planes read (window sums)
  const double* fin2;    // K_ADJ_GATHER: window sums of the averaging fields
  double* fout;          // FP64 field planes written
  double* red;           // K_ADJ_SOLVE: per-workgroup sums of dL/deps, dL/deps_mul
  float* out2;           // K_ADJ_GATHER: dL/d(noisy)
  int average;
  // downsampled-moment variant only
  int block, Hl, Wl, lr_R;
  int lr_rows;  // K_LR_APPLY: full-resolution rows per workgroup (0: one lane per pixel)
  // batched launches (K_COEFFS_BATCH, K_APPLY_AVG_BATCH, K_UP_APPLY_BATCH):
  // workgroup b belongs to the frame f with wg_start[f] <= b < wg_start[f + 1]
  // and runs as workgroup b - wg_start[f] of frames[f]
  const struct LaunchArgs* frames;
  const int* wg_start;
  const BatchPlanDev* bplan;  // K_BATCH_PERSISTENT
  int nframes;
  int batch_blocks;  // total workgroups of the launch
  int up;            // K_UP_APPLY: upsampling factor (coefficient grid = H / up)
  const float* guides_low;  // K_UP_APPLY: the guides the models were fitted on (anchors)
  double taps[2 * kMaxLowresRadius + 1];
};

// LDS of the staged model interpolation: rows x models x low-resolution
// columns of FP64 (a workgroup's kThreads columns span at most
// (kThreads - 1) / block + 3 low-resolution columns).
inline size_t lr_apply_lds_bytes(int Q, int C, int block, int rows) {
  return (size_t)rows * (Q + 1) * C * ((kThreads - 1) / block + 3) * sizeof(double);
}
// Rows per workgroup of the staged interpolation: the most of 8, 4, 2, 1
// whose staging fits in 64 KiB; 0 when none does (one lane per pixel then).
inline int lr_apply_rows(int Q, int C, int block) {
  for (int rows = 8; rows >= 1; rows /= 2)
    if (lr_apply_lds_bytes(Q, C, block, rows) <= 65536) return rows;
  return 0;
}

// The downsampled-moment variant's low-resolution planes: the pixel count
// n then the num_sums(Q, C) anchored product sums (FP64, [planes][Hl][Wl]);
// models b~ (C) then a (Q*C) in anchored units (FP64).
// dst[p][I][J] = sum_{|d|, |e| <= R} taps[d + R] taps[e + R] src[p][I + d][J + e]
// (zero outside the grid): the separable low-resolution blur.
hipError_t launch_lr_blur(const double* src, double* dst, int planes, int Hl, int Wl, int R,
                          const double* taps, hipStream_t s);

// Adjoint field planes (FP64, [planes][H][W]).
//  averaging fields: G_c / n (C), g~_q G_c / n (Q*C), a_qc (Q*C) (K_ADJ_COEF
//  writes the a_qc; the window-sum pass forms the others from the inputs);
//  solve fields, K_ADJ_SOLVE: 2 dW / n (upper triangle), Gv / n (Q*C),
//  e (Q), f (C) -- num_sums(Q, C) planes.
__host__ __device__ constexpr int num_avg_fields(int Q, int C) { return C + 2 * Q * C; }

// FP64 clipped window sums of `planes` planes of H x W (separable: running
// column sums, then a row pass through LDS). src and dst must not overlap.
hipError_t launch_box(const double* src, double* dst, int planes, int H, int W, int r,
                      hipStream_t s);
// FP32 window means (clipped window, FP64 sums) of `planes` planes of H x W.
hipError_t launch_mean_planes(const float* src, float* dst, int planes, int H, int W, int r,
                              hipStream_t s);
// The same for FP64 planes, FP64 means.
hipError_t launch_mean_planes64(const double* src, double* dst, int planes, int H, int W, int r,
                                hipStream_t s);
// FP64 clipped window sums of the num_sums(Q, C) anchored products of the
// inputs, in the moment order g_q | y_c | g_p g_q (p <= q) | g_q y_c, each
// input plane shifted by its value at pixel (0, 0).
// With with_count, plane 0 is the window pixel count and the channels follow
// (the plane order of the downsampled-moment variant's solve).
hipError_t launch_box_products(const float* guides, const float* noisy, int Q, int C, int H,
                               int W, int r, double* dst, hipStream_t s,
                               bool with_count = false);
// FP64 clipped window sums of the adjoint's averaging products, formed from
// the inputs: G_c / n (C planes) then g~_q G_c / n (Q*C planes), with G =
// dL/d(output), n the pixel's window count and g~ each guide shifted by its
// value at pixel (0, 0).
hipError_t launch_box_avgfields(const float* guides, const float* gout, int Q, int C, int H,
                                int W, int r, double* dst, hipStream_t s);
// dst[0..1] = sums over n entries of the interleaved pairs src[2i], src[2i+1]
// (fixed order; one workgroup).
hipError_t launch_pair_sum(const double* src, int n, double* dst, hipStream_t s);

__host__ __device__ constexpr int num_sums(int Q, int C) {
  return Q + C + Q * (Q + 1) / 2 + Q * C;
}

// Output columns per strip for a walker kernel.
inline int strip_out_cols(int kind, int r) {
  if (kind == K_FUSED1) return kThreads - 4 * r;
  return kThreads - 2 * r;  // K_MOMENTS, K_FUSED0, K_APPLY_AVG
}

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Output rows per tile of the coefficient-averaging kernel (sizes its
// per-lane register arrays and its LDS), and the workgroups of it that
// registers and LDS let a CU hold.
#ifndef FLR_AVG_TILE_ROWS
#define FLR_AVG_TILE_ROWS 17
#endif
constexpr int kAvgTileRows = FLR_AVG_TILE_ROWS;
constexpr int kAvgPerCU = kAvgTileRows <= 8 ? 4 : (kAvgTileRows <= 12 ? 3 : 2);

// XCDs of the GPU (workgroups are dealt to them round-robin), and the
// workgroups of an averaging launch over `tiles` tiles: whole rounds of the
// XCDs, so that each XCD runs a contiguous run of tiles (apply_avg_kernel).
constexpr int kXcds = 8;
inline int avg_groups(int tiles) { return (tiles + kXcds - 1) / kXcds * kXcds; }

// Workgroups of a walker kernel resident per CU (the coefficient-averaging
// kernel's kAvgPerCU, one for the others).
inline int workgroups_per_cu(int kind) { return kind == K_APPLY_AVG ? kAvgPerCU : 1; }

// Rows of coefficient halo a walker recomputes above and below its segment.
inline int row_halo(int kind, int r) { return kind == K_FUSED1 ? r : 0; }

// Pick tiles and segments. With tile_rows > 0 the caller fixes the segment
// length; otherwise minimise (workgroup waves) x (rows walked per segment).
// K_MOMENTS, K_FUSED0, K_COEFFS and K_APPLY_AVG have no coefficient-row halo.
inline void plan_walk(int kind, int H, int W, int r, int tile_rows, int* tiles_x, int* n_seg,
                      int* seg_rows) {
  const int tout = strip_out_cols(kind, r);
  *tiles_x = ceil_div(W, tout);
  const int rmax = kind == K_APPLY_AVG ? kAvgTileRows : H;
  if (tile_rows > 0) {
    int t = tile_rows < H ? tile_rows : H;
    *seg_rows = t < rmax ? t : rmax;
    *n_seg = ceil_div(H, *seg_rows);
    return;
  }
  if (kind == K_APPLY_AVG) {
    // every tile reads its rows plus 2r halo rows of each coefficient plane
    double best = 1e300;
    int best_n = ceil_div(H, rmax);
    for (int n = best_n; n <= H; ++n) {
      const int R = ceil_div(H, n);
      if (n > best_n && ceil_div(H, n - 1) == R) continue;
      const double waves = (double)ceil_div(*tiles_x * n, kCUs * workgroups_per_cu(kind));
      const double cost = waves * (double)(R + 2 * r) + 1e-3 * n;
      if (cost < best) {
        best = cost;
        best_n = n;
      }
    }
    *n_seg = best_n;
    *seg_rows = ceil_div(H, best_n);
    return;
  }
  const int hc = row_halo(kind, r);
  const int per_cu = workgroups_per_cu(kind);
  double best = 1e300;
  int best_n = 1;
  const int nmax = H < 4096 ? H : 4096;
  for (int n = 1; n <= nmax; ++n) {
    const int R = ceil_div(H, n);
    if (n > 1 && ceil_div(H, n - 1) == R) continue;
    const int wgs = *tiles_x * n;
    const double waves = (double)ceil_div(wgs, kCUs * per_cu);
    // rows solved per segment plus a share for the moment warm-up rows
    const double cost = waves * ((double)R + 2.0 * hc + 0.5 * r) + 1e-3 * n;
    if (cost < best) {
      best = cost;
      best_n = n;
    }
  }
  *seg_rows = ceil_div(H, best_n);
  *n_seg = ceil_div(H, *seg_rows);
}

// Chunk length for the LDS horizontal pass over `rows` channel rows and
// `nout` outputs: minimise (task passes) x (window taps + 2 per output). A
// pass runs two tasks per thread side by side, so its latency is that of one.
inline int plan_chunk(int rows, int nout, int r) {
  int best = nout;
  double bestc = 1e300;
  for (int nch = 1; nch <= nout; ++nch) {
    const int chunk = ceil_div(nout, nch);
    if (nch > 1 && ceil_div(nout, nch - 1) == chunk) continue;
    const int passes = ceil_div(rows * ceil_div(nout, chunk), 2 * kThreads);
    const double cost = passes * (2.0 * r + 1 + 2.0 * (chunk - 1));
    if (cost < bestc) {
      bestc = cost;
      best = chunk;
    }
  }
  return best;
}

// LDS layout of the walker kernels (bytes, rows of kLdsStride elements):
//   [0, a)            source rows of the horizontal pass (one moment group);
//   [a, a + b)        destination rows (moment group, or coefficient sums);
//   [a + b, + va)     K_FUSED1 only, when it fits: the persistent vertical
//                     window sums of the coefficients, F*C rows of solve_t,
//                     read directly by the horizontal averaging pass.
// Moment channels are processed in groups of `mg` rows; the first group
// always holds all Q + C first moments.
struct WalkLayout {
  int mg;          // moment rows per group
  int ag;          // coefficient rows per averaging group (va_lds: all F*C)
  bool va_lds;     // coefficient sums live in LDS
  size_t a, b, va; // region sizes in bytes
};

__host__ __device__ constexpr WalkLayout walk_layout(int Q, int C, int kind, int ns_walk = -1) {
  const int ns = ns_walk > 0 ? ns_walk : num_sums(Q, C);
  const int fc = (Q + 1) * C;
  const int row_s = kLdsStride * (int)sizeof(sum_t);
  const int row_t = kLdsStride * (int)sizeof(solve_t);
  WalkLayout L{0, 0, false, 0, 0, 0};
  if (kind == K_APPLY_AVG) {
    // two buffers of segment prefixes, one row per output row of the tile
    L.ag = fc;
    L.a = L.b = (size_t)kAvgTileRows * row_t;
    return L;
  }
  if (kind == K_FUSED1) {
    const int va = fc * row_t;
    const int left = kLdsBytes - 2 * va;  // Va region + destination sized for F*C rows
    const int mg_max = left > 0 ? left / row_s : 0;
    if (mg_max >= Q + C) {
      const int ng = (ns + mg_max - 1) / mg_max;
      L.mg = (ns + ng - 1) / ng;
      L.ag = fc;
      L.va_lds = true;
      L.a = (size_t)L.mg * row_s;
      const size_t bm = (size_t)L.mg * row_s;
      L.b = bm > (size_t)va ? bm : (size_t)va;
      L.va = (size_t)va;
      return L;
    }
  }
  L.mg = group_size(ns, sizeof(sum_t));
  L.ag = group_size(fc, sizeof(solve_t));
  const size_t m = (size_t)L.mg * row_s;
  const size_t c = (size_t)L.ag * row_t;
  L.a = L.b = m > c ? m : c;
  return L;
}

inline size_t walk_lds_bytes(int kind, int Q, int C, int ns_walk = -1) {
  const WalkLayout L = walk_layout(Q, C, kind, ns_walk);
  return L.a + L.b + L.va;
}

// LDS of the persistent batch kernel: the larger of the walk's and the
// averaging kernel's (its box items use the ring where it fits in that).
inline size_t batch_lds_bytes(int Q, int C) {
  const size_t w = walk_lds_bytes(K_COEFFS, Q, C), v = walk_lds_bytes(K_APPLY_AVG, Q, C);
  return w > v ? w : v;
}

// Split walks: when a moment walker's channels exceed what stays resident in
// LDS between rows (two groups of max_lds_rows FP64 rows for 256 columns),
// the product channels are walked in two slices, each with the first
// moments: [0, split_first) then the rest. Only where both slices fit.
__host__ __device__ constexpr int num_products(int Q, int C) { return Q * (Q + 1) / 2 + Q * C; }
__host__ __device__ constexpr int resident_channels() { return 2 * max_lds_rows(8); }
__host__ __device__ constexpr int split_first(int Q, int C) { return (num_products(Q, C) + 1) / 2; }
__host__ __device__ constexpr bool split_walk(int Q, int C) {
  return num_sums(Q, C) > resident_channels() &&
         Q + C + split_first(Q, C) <= resident_channels();
}

inline size_t ring_bytes_per_block(int Q, int C, int r) {
  return (size_t)(2 * r + 1) * (Q + 1) * C * kThreads * sizeof(ring_t);
}

// Per-guide-count dispatch entry points (one translation unit each).
#define FLR_DECLARE_Q(q) \
  hipError_t launch_q##q(int C, int kind, const LaunchArgs& a, hipStream_t s);
FLR_DECLARE_Q(1)
FLR_DECLARE_Q(2)
FLR_DECLARE_Q(3)
FLR_DECLARE_Q(4)
FLR_DECLARE_Q(5)
FLR_DECLARE_Q(6)
FLR_DECLARE_Q(7)
FLR_DECLARE_Q(8)
FLR_DECLARE_Q(9)
FLR_DECLARE_Q(10)
FLR_DECLARE_Q(11)
FLR_DECLARE_Q(12)
#undef FLR_DECLARE_Q

}  // namespace flr
