// Host side of the C ABI declared in include/flr.h: argument validation
// (pure CPU, before any HIP call), launch planning and dispatch to the
// per-guide-count kernel instantiations.
#include <math.h>
#include <initializer_list>
#include <stdint.h>

#include "flr.h"
#include "flr_launch.hpp"

namespace {

using flr::LaunchArgs;

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
  return a0 < b0 + nb && b0 < a0 + na;
}

size_t plane_bytes(const flr_params* p) {
  return (size_t)p->height * (size_t)p->width * sizeof(float);
}

flr_status check_ptrs(std::initializer_list<const void*> ptrs) {
  for (const void* q : ptrs)
    if (!q) return FLR_ERR_NULL;
  for (const void* q : ptrs)
    if (!aligned16(q)) return FLR_ERR_ALIGN;
  return FLR_OK;
}

LaunchArgs base_args(const flr_params* p) {
  LaunchArgs a = {};
  a.H = p->height;
  a.W = p->width;
  a.r = p->radius;
  a.eps = p->eps;
  a.eps_mul = p->eps_mul;
  a.eps_dev = p->eps_device;
  a.reg_mode = p->reg_mode;
  a.raw = (p->flags & FLR_FLAG_RAW_MOMENTS) ? 1 : 0;
  return a;
}

void plan(const flr_params* p, int kind, LaunchArgs* a) {
  flr::plan_walk(kind, p->height, p->width, p->radius, p->tile_rows, &a->tiles_x, &a->n_seg,
                 &a->seg_rows);
  const int Q = p->num_guides, C = p->num_channels, r = p->radius;
  const int ncoef = flr::kThreads - 2 * r;
  const flr::WalkLayout L = flr::walk_layout(Q, C, kind);
  a->hchunk_m = L.mg > 0 ? flr::plan_chunk(L.mg, ncoef, r) : 1;
  a->hchunk_a = flr::plan_chunk(L.ag, flr::strip_out_cols(kind, r), r);
}

flr_status dispatch(int Q, int C, int kind, const LaunchArgs& a, void* stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e;
  switch (Q) {
    case 1: e = flr::launch_q1(C, kind, a, s); break;
    case 2: e = flr::launch_q2(C, kind, a, s); break;
    case 3: e = flr::launch_q3(C, kind, a, s); break;
    case 4: e = flr::launch_q4(C, kind, a, s); break;
    case 5: e = flr::launch_q5(C, kind, a, s); break;
    case 6: e = flr::launch_q6(C, kind, a, s); break;
    case 7: e = flr::launch_q7(C, kind, a, s); break;
    case 8: e = flr::launch_q8(C, kind, a, s); break;
    case 9: e = flr::launch_q9(C, kind, a, s); break;
    case 10: e = flr::launch_q10(C, kind, a, s); break;
    case 11: e = flr::launch_q11(C, kind, a, s); break;
    case 12: e = flr::launch_q12(C, kind, a, s); break;
    default: return FLR_ERR_CHANNELS;
  }
  return e == hipSuccess ? FLR_OK : FLR_ERR_HIP;
}

size_t ring_bytes(const flr_params* p) {
  int tiles_x, n_seg, seg_rows;
  flr::plan_walk(flr::K_FUSED1, p->height, p->width, p->radius, p->tile_rows, &tiles_x, &n_seg,
                 &seg_rows);
  return (size_t)tiles_x * n_seg *
         flr::ring_bytes_per_block(p->num_guides, p->num_channels, p->radius);
}

// Unfused workspace: the moment image, then the coefficient image at the
// next 256-byte boundary.
// Bytes of a coefficient image: (Q + 1) C planes, plus C with the intercept
// pair's lo parts.
size_t coeff_image_bytes(const flr_params* p) {
  const size_t planes = (size_t)(p->num_guides + 1) * p->num_channels +
                        ((p->flags & FLR_FLAG_INTERCEPT_PAIR) ? p->num_channels : 0);
  return planes * (size_t)p->height * p->width * sizeof(float);
}

size_t unfused_coeff_offset(const flr_params* p) {
  const size_t mb = flr_num_moment_planes(p->num_guides, p->num_channels) * plane_bytes(p);
  return (mb + 255) / 256 * 256;
}

// Workspace of flr_denoise_backward, byte offsets of 256-aligned FP64
// regions: the window sums of the anchored input products (later reused for
// the window sums of the solve fields), the coefficients a, the window sums
// of the averaging fields (with averaging only: the averaging products and
// a), the solve fields, and the per-workgroup sums of the regulariser
// gradients.
struct BackwardLayout {
  size_t sums, f1, s1, f2, red, total;
};

BackwardLayout backward_layout(const flr_params* p) {
  const int Q = p->num_guides, C = p->num_channels;
  const size_t pl = (size_t)p->height * p->width;
  const size_t pblocks = (pl + 255) / 256;
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t ns = (size_t)flr::num_sums(Q, C), ns1 = (size_t)flr::num_avg_fields(Q, C);
  BackwardLayout L{};
  size_t o = 0;
  L.sums = o;
  o += al(ns * pl * sizeof(double));
  L.f1 = o;
  o += al((size_t)Q * C * pl * sizeof(double));
  L.s1 = o;
  if (p->average_coeffs) o += al(ns1 * pl * sizeof(double));
  L.f2 = o;
  o += al(ns * pl * sizeof(double));
  L.red = o;
  o += al(2 * pblocks * sizeof(double));
  L.total = o;
  return L;
}

// Workspace of flr_denoise_lowres: FP64 low-resolution planes, the block
// sums (count + num_sums channels), their row-blurred copy and the models.
struct LowresLayout {
  int Hl, Wl;
  size_t sums, tmp, coef, total;
};

LowresLayout lowres_layout(const flr_params* p, int block) {
  const int Q = p->num_guides, C = p->num_channels;
  LowresLayout L{};
  L.Hl = (p->height + block - 1) / block;
  L.Wl = (p->width + block - 1) / block;
  const size_t pll = (size_t)L.Hl * L.Wl;
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t np = 1 + (size_t)flr::num_sums(Q, C);
  size_t o = 0;
  L.sums = o;
  o += al(np * pll * sizeof(double));
  L.tmp = o;
  o += al(np * pll * sizeof(double));
  L.coef = o;
  o += al((size_t)(Q + 1) * C * pll * sizeof(double));
  L.total = o;
  return L;
}

flr_status validate_lowres(const flr_params* p, int block, float sigma, int radius_low) {
  flr_status st = flr_validate_params(p);
  if (st != FLR_OK) return st;
  if (block < 1 || block > 16 || (block & (block - 1))) return FLR_ERR_MODE;
  if (!isfinite(sigma) || sigma < 0.f) return FLR_ERR_EPS;
  if (radius_low < 0 || radius_low > flr::kMaxLowresRadius) return FLR_ERR_RADIUS;
  if (p->flags) return FLR_ERR_MODE;
  return FLR_OK;
}

// Workspace of a batch: the launch tables, then per frame its coefficient
// image on the noisy grid, then per joint frame its averaged coefficients.
struct BatchLayout {
  // coef: a plain frame's coefficient image, or a joint frame's FP64 sums;
  // the persistent launch's tables: launch arguments (largs), box-pass
  // arguments (bargs), stages, its header (pdev), control words and counters
  size_t walk, apply, up, starts, largs, bargs, stages, pdev, ctl, counters, ncounters,
      coef[FLR_BATCH_MAX], models[FLR_BATCH_MAX], mean[FLR_BATCH_MAX], total;
};

bool frame_is_joint(const flr_frame& f) { return f.guides_low != nullptr; }

int frame_up(const flr_frame& f) {
  return f.noisy_height > 0 ? f.height / f.noisy_height : 0;
}

BatchLayout batch_layout(const flr_params* p, const flr_frame* frames, int n) {
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  BatchLayout L{};
  const size_t fc = (size_t)(p->num_guides + 1) * p->num_channels;
  size_t o = 0;
  L.walk = o;
  o += al(n * sizeof(LaunchArgs));
  L.apply = o;
  o += al(n * sizeof(LaunchArgs));
  L.up = o;
  o += al(n * sizeof(LaunchArgs));
  L.starts = o;
  o += al(3 * (n + 1) * sizeof(int));
  L.largs = o;
  o += al(4 * n * sizeof(LaunchArgs));
  L.bargs = o;
  o += al(2 * n * sizeof(flr::AdjBoxArgs));
  L.stages = o;
  o += al(4 * n * sizeof(flr::BatchStage));
  L.pdev = o;
  o += al(sizeof(flr::BatchPlanDev));
  L.ctl = o;
  o += al(4 * sizeof(int));
  // at most one counter per row of each frame's walk, three per joint frame
  L.ncounters = 3 * (size_t)n;
  for (int i = 0; i < n; ++i) L.ncounters += (size_t)frames[i].noisy_height;
  L.counters = o;
  o += al(L.ncounters * sizeof(int));
  const size_t ns1 = 1 + (size_t)flr::num_sums(p->num_guides, p->num_channels);
  for (int i = 0; i < n; ++i) {
    const size_t px = (size_t)frames[i].noisy_height * frames[i].noisy_width;
    L.coef[i] = o;
    if (!frame_is_joint(frames[i])) {  // b (hi), a, b (lo): as flr_denoise's two-pass path
      o += al((fc + p->num_channels) * px * sizeof(float));
    } else {  // sums, models, means
      o += al(ns1 * px * sizeof(double));
      L.models[i] = o;
      o += al(fc * px * sizeof(double));
      L.mean[i] = o;
      o += al(fc * px * sizeof(double));
    }
  }
  L.total = o;
  return L;
}

flr_status validate_batch(const flr_params* p, const flr_frame* frames, int n) {
  if (!p || !frames) return FLR_ERR_NULL;
  if (n < 1 || n > FLR_BATCH_MAX) return FLR_ERR_SHAPE;
  flr_params q = *p;
  q.height = q.width = 1;
  flr_status st = flr_validate_params(&q);
  if (st != FLR_OK) return st;
  if (!p->average_coeffs || p->flags) return FLR_ERR_MODE;
  if (flr::split_walk(p->num_guides, p->num_channels) ||
      flr::num_sums(p->num_guides, p->num_channels) > flr::resident_channels())
    return FLR_ERR_CHANNELS;
  const int Q = p->num_guides, C = p->num_channels;
  for (int i = 0; i < n; ++i) {
    const flr_frame& f = frames[i];
    q.height = f.height;
    q.width = f.width;
    if ((st = flr_validate_params(&q)) != FLR_OK) return st;
    if (f.noisy_height < 1 || f.noisy_width < 1 || f.tile_rows < 0 || f.apply_rows < 0)
      return FLR_ERR_SHAPE;
    if (frame_is_joint(f)) {
      const int up = frame_up(f);
      if ((up != 2 && up != 4 && up != 8) || f.height != up * f.noisy_height ||
          f.width != up * f.noisy_width)
        return FLR_ERR_SHAPE;
    } else if (f.noisy_height != f.height || f.noisy_width != f.width) {
      return FLR_ERR_SHAPE;
    }
    if ((st = check_ptrs({f.guides, f.noisy, f.out})) != FLR_OK) return st;
    if (frame_is_joint(f) && !aligned16(f.guides_low)) return FLR_ERR_ALIGN;
  }
  // outputs against every input and every other output
  for (int i = 0; i < n; ++i) {
    const size_t ob = (size_t)C * frames[i].height * frames[i].width * sizeof(float);
    for (int j = 0; j < n; ++j) {
      const flr_frame& g = frames[j];
      const size_t gb = (size_t)Q * g.height * g.width * sizeof(float);
      const size_t nb = (size_t)C * g.noisy_height * g.noisy_width * sizeof(float);
      const size_t lb = (size_t)Q * g.noisy_height * g.noisy_width * sizeof(float);
      if (overlaps(frames[i].out, ob, g.guides, gb) || overlaps(frames[i].out, ob, g.noisy, nb) ||
          (g.guides_low && overlaps(frames[i].out, ob, g.guides_low, lb)))
        return FLR_ERR_ALIAS;
      if (j != i && overlaps(frames[i].out, ob, g.out,
                             (size_t)C * g.height * g.width * sizeof(float)))
        return FLR_ERR_ALIAS;
    }
  }
  return FLR_OK;
}

}  // namespace

extern "C" {

size_t flr_num_moment_planes(int32_t Q, int32_t C) {
  if (Q < 1 || Q > FLR_MAX_GUIDES || C < 1 || C > FLR_MAX_CHANNELS) return 0;
  return (size_t)(1 + flr::num_sums(Q, C));
}

size_t flr_num_coeff_planes(int32_t Q, int32_t C) {
  if (Q < 1 || Q > FLR_MAX_GUIDES || C < 1 || C > FLR_MAX_CHANNELS) return 0;
  return (size_t)(Q + 1) * C;
}

flr_status flr_validate_params(const flr_params* p) {
  if (!p) return FLR_ERR_NULL;
  if (p->height < 1 || p->width < 1 || p->height > FLR_MAX_DIM || p->width > FLR_MAX_DIM)
    return FLR_ERR_SHAPE;
  if ((int64_t)p->height * p->width > ((int64_t)1 << 28)) return FLR_ERR_SHAPE;
  if (p->num_guides < 1 || p->num_guides > FLR_MAX_GUIDES || p->num_channels < 1 ||
      p->num_channels > FLR_MAX_CHANNELS)
    return FLR_ERR_CHANNELS;
  if (p->radius < 0 || p->radius > FLR_MAX_RADIUS) return FLR_ERR_RADIUS;
  if (!isfinite(p->eps) || p->eps < 0.f || !isfinite(p->eps_mul) || p->eps_mul < 0.f)
    return FLR_ERR_EPS;
  if (p->reg_mode != FLR_REG_RIDGE && p->reg_mode != FLR_REG_PAPER) return FLR_ERR_MODE;
  if ((p->average_coeffs != 0 && p->average_coeffs != 1) || p->fused < 0 || p->fused > 2)
    return FLR_ERR_MODE;
  if (p->flags & ~(uint32_t)(FLR_FLAG_RAW_MOMENTS | FLR_FLAG_INTERCEPT_PAIR)) return FLR_ERR_MODE;
  if (p->tile_rows < 0) return FLR_ERR_SHAPE;
  if (reinterpret_cast<uintptr_t>(p->eps_device) & 3u) return FLR_ERR_ALIGN;
  return FLR_OK;
}

size_t flr_denoise_workspace_bytes(const flr_params* p) {
  if (flr_validate_params(p) != FLR_OK) return 0;
  const size_t pb = plane_bytes(p);
  if (p->fused == FLR_PATH_STAGES)
    return unfused_coeff_offset(p) + flr_num_coeff_planes(p->num_guides, p->num_channels) * pb;
  if (!p->average_coeffs) return 0;
  // the two-pass path's coefficient image: b (hi), a, then b (lo)
  const size_t cb = (flr_num_coeff_planes(p->num_guides, p->num_channels) + p->num_channels) * pb;
  if (p->fused == FLR_PATH_TWO_PASS && !flr::split_walk(p->num_guides, p->num_channels))
    return cb;
  if (p->fused == FLR_PATH_TWO_PASS)  // split walks: first slice's moment planes, coefficients
    return unfused_coeff_offset(p) + cb;
  return ring_bytes(p);
}

flr_status flr_moments(const flr_params* p, const float* guides, const float* noisy,
                       float* moments, void* stream) {
  flr_status st = flr_validate_params(p);
  if (st != FLR_OK) return st;
  if ((st = check_ptrs({guides, noisy, moments})) != FLR_OK) return st;
  const size_t pb = plane_bytes(p);
  const size_t mb = flr_num_moment_planes(p->num_guides, p->num_channels) * pb;
  if (overlaps(moments, mb, guides, p->num_guides * pb) ||
      overlaps(moments, mb, noisy, p->num_channels * pb))
    return FLR_ERR_ALIAS;
  LaunchArgs a = base_args(p);
  a.guides = guides;
  a.noisy = noisy;
  a.out = moments;
  plan(p, flr::K_MOMENTS, &a);
  if (flr::split_walk(p->num_guides, p->num_channels)) {
    // two walks over halves of the product channels, each LDS-resident
    if ((st = dispatch(p->num_guides, p->num_channels, flr::K_MOMENTS_A, a, stream)) != FLR_OK)
      return st;
    return dispatch(p->num_guides, p->num_channels, flr::K_MOMENTS_B, a, stream);
  }
  return dispatch(p->num_guides, p->num_channels, flr::K_MOMENTS, a, stream);
}

flr_status flr_solve(const flr_params* p, const float* moments, float* coeffs, void* stream) {
  flr_status st = flr_validate_params(p);
  if (st != FLR_OK) return st;
  if ((st = check_ptrs({moments, coeffs})) != FLR_OK) return st;
  if (p->flags & FLR_FLAG_INTERCEPT_PAIR) return FLR_ERR_MODE;
  const size_t pb = plane_bytes(p);
  if (overlaps(coeffs, flr_num_coeff_planes(p->num_guides, p->num_channels) * pb, moments,
               flr_num_moment_planes(p->num_guides, p->num_channels) * pb))
    return FLR_ERR_ALIAS;
  LaunchArgs a = base_args(p);
  a.planes = moments;
  a.out = coeffs;
  return dispatch(p->num_guides, p->num_channels, flr::K_SOLVE, a, stream);
}

flr_status flr_coefficients(const flr_params* p, const float* guides, const float* noisy,
                            float* coeffs, void* stream) {
  flr_status st = flr_validate_params(p);
  if (st != FLR_OK) return st;
  if ((st = check_ptrs({guides, noisy, coeffs})) != FLR_OK) return st;
  if (p->flags & FLR_FLAG_RAW_MOMENTS) return FLR_ERR_MODE;
  const size_t pb = plane_bytes(p);
  const size_t cb = coeff_image_bytes(p);
  if (overlaps(coeffs, cb, guides, p->num_guides * pb) ||
      overlaps(coeffs, cb, noisy, p->num_channels * pb))
    return FLR_ERR_ALIAS;
  LaunchArgs a = base_args(p);
  a.guides = guides;
  a.noisy = noisy;
  a.out = coeffs;
  a.coef_lo = (p->flags & FLR_FLAG_INTERCEPT_PAIR) ? 1 : 0;
  plan(p, flr::K_COEFFS, &a);
  return dispatch(p->num_guides, p->num_channels, flr::K_COEFFS, a, stream);
}

flr_status flr_apply(const flr_params* p, const float* guides, const float* coeffs, float* out,
                     void* stream) {
  flr_status st = flr_validate_params(p);
  if (st != FLR_OK) return st;
  if ((st = check_ptrs({guides, coeffs, out})) != FLR_OK) return st;
  const size_t pb = plane_bytes(p);
  const size_t ob = p->num_channels * pb;
  if (overlaps(out, ob, guides, p->num_guides * pb) ||
      overlaps(out, ob, coeffs, coeff_image_bytes(p)))
    return FLR_ERR_ALIAS;
  LaunchArgs a = base_args(p);
  a.guides = guides;
  a.planes = coeffs;
  a.out = out;
  a.coef_lo = (p->flags & FLR_FLAG_INTERCEPT_PAIR) ? 1 : 0;
  const int kind = p->average_coeffs ? flr::K_APPLY_AVG : flr::K_APPLY_POINT;
  if (kind == flr::K_APPLY_AVG) plan(p, kind, &a);
  return dispatch(p->num_guides, p->num_channels, kind, a, stream);
}

flr_status flr_denoise(const flr_params* p_in, const float* guides, const float* noisy,
                       float* out, void* workspace, size_t workspace_bytes, void* stream) {
  flr_status st = flr_validate_params(p_in);
  if (st != FLR_OK) return st;
  // the intercept-pair flag has no effect here (the two-pass path always
  // keeps the pair, the stage sequence never)
  flr_params pc = *p_in;
  pc.flags &= ~(uint32_t)FLR_FLAG_INTERCEPT_PAIR;
  const flr_params* p = &pc;
  if ((st = check_ptrs({guides, noisy, out})) != FLR_OK) return st;
  if (p->flags & FLR_FLAG_RAW_MOMENTS) return FLR_ERR_MODE;
  const size_t pb = plane_bytes(p);
  const size_t ob = p->num_channels * pb;
  if (overlaps(out, ob, guides, p->num_guides * pb) ||
      overlaps(out, ob, noisy, p->num_channels * pb))
    return FLR_ERR_ALIAS;
  const size_t need = flr_denoise_workspace_bytes(p);
  if (need > 0) {
    if (!workspace || workspace_bytes < need) return FLR_ERR_WORKSPACE;
    if (!aligned16(workspace)) return FLR_ERR_ALIGN;
    if (overlaps(workspace, need, guides, p->num_guides * pb) ||
        overlaps(workspace, need, noisy, p->num_channels * pb) ||
        overlaps(workspace, need, out, ob))
      return FLR_ERR_ALIAS;
  }
  const int Q = p->num_guides, C = p->num_channels;
  // two-pass: the coefficient image with hi + lo intercepts (LaunchArgs::coef_lo)
  auto apply_lo = [&](const float* coeffs) {
    LaunchArgs a = base_args(p);
    a.guides = guides;
    a.planes = coeffs;
    a.out = out;
    a.coef_lo = 1;
    plan(p, flr::K_APPLY_AVG, &a);
    return dispatch(Q, C, flr::K_APPLY_AVG, a, stream);
  };
  if (p->fused == FLR_PATH_TWO_PASS && p->average_coeffs && !flr::split_walk(Q, C)) {
    float* coeffs = static_cast<float*>(workspace);
    LaunchArgs a = base_args(p);
    a.guides = guides;
    a.noisy = noisy;
    a.out = coeffs;
    a.coef_lo = 1;
    plan(p, flr::K_COEFFS, &a);
    if ((st = dispatch(Q, C, flr::K_COEFFS, a, stream)) != FLR_OK) return st;
    return apply_lo(coeffs);
  }
  if (p->fused == FLR_PATH_TWO_PASS && p->average_coeffs) {
    // Too many moment channels for one LDS-resident walk: the walk over the
    // first slice of the product channels writes its moment planes, the
    // walk over the second reads them back at each pixel and solves there
    // (no second slice of planes, no separate solve), then the averaging.
    float* moments = static_cast<float*>(workspace);
    float* coeffs =
        reinterpret_cast<float*>(static_cast<char*>(workspace) + unfused_coeff_offset(p));
    LaunchArgs a = base_args(p);
    a.guides = guides;
    a.noisy = noisy;
    a.out = moments;
    plan(p, flr::K_MOMENTS, &a);
    if ((st = dispatch(Q, C, flr::K_MOMENTS_A, a, stream)) != FLR_OK) return st;
    LaunchArgs b = base_args(p);
    b.guides = guides;
    b.noisy = noisy;
    b.planes = moments;
    b.out = coeffs;
    b.coef_lo = 1;
    plan(p, flr::K_COEFFS, &b);
    if ((st = dispatch(Q, C, flr::K_SPLIT_COEFFS, b, stream)) != FLR_OK) return st;
    return apply_lo(coeffs);
  }
  // The stage sequence (its moment walk split into two slices when there
  // are too many moment channels for one LDS-resident walk).
  const bool stages = p->fused == FLR_PATH_STAGES;
  if (!stages) {
    LaunchArgs a = base_args(p);
    a.guides = guides;
    a.noisy = noisy;
    a.out = out;
    a.ring = static_cast<float*>(workspace);
    const int kind = p->average_coeffs ? flr::K_FUSED1 : flr::K_FUSED0;
    plan(p, kind, &a);
    return dispatch(Q, C, kind, a, stream);
  }
  float* moments = static_cast<float*>(workspace);
  float* coeffs = reinterpret_cast<float*>(static_cast<char*>(workspace) + unfused_coeff_offset(p));
  if ((st = flr_moments(p, guides, noisy, moments, stream)) != FLR_OK) return st;
  if ((st = flr_solve(p, moments, coeffs, stream)) != FLR_OK) return st;
  return flr_apply(p, guides, coeffs, out, stream);
}

size_t flr_denoise_backward_workspace_bytes(const flr_params* p) {
  if (flr_validate_params(p) != FLR_OK) return 0;
  return backward_layout(p).total;
}

flr_status flr_denoise_backward(const flr_params* p, const float* guides, const float* noisy,
                                const float* grad_out, float* grad_guides, float* grad_noisy,
                                double* grad_reg, void* workspace, size_t workspace_bytes,
                                void* stream) {
  flr_status st = flr_validate_params(p);
  if (st != FLR_OK) return st;
  if ((st = check_ptrs({guides, noisy, grad_out, grad_guides, grad_noisy})) != FLR_OK) return st;
  if (grad_reg && !aligned16(grad_reg)) return FLR_ERR_ALIGN;
  if (p->flags) return FLR_ERR_MODE;
  const BackwardLayout L = backward_layout(p);
  if (!workspace || workspace_bytes < L.total) return FLR_ERR_WORKSPACE;
  if (!aligned16(workspace)) return FLR_ERR_ALIGN;
  const int Q = p->num_guides, C = p->num_channels;
  const size_t pb = plane_bytes(p);
  const void* ins[3] = {guides, noisy, grad_out};
  const size_t nin[3] = {Q * pb, C * pb, C * pb};
  const void* outs[4] = {grad_guides, grad_noisy, grad_reg, workspace};
  const size_t nout[4] = {Q * pb, C * pb, grad_reg ? 2 * sizeof(double) : 0, L.total};
  for (int o = 0; o < 4; ++o) {
    if (!nout[o]) continue;
    for (int i = 0; i < 3; ++i)
      if (overlaps(outs[o], nout[o], ins[i], nin[i])) return FLR_ERR_ALIAS;
    for (int o2 = o + 1; o2 < 4; ++o2)
      if (nout[o2] && overlaps(outs[o], nout[o], outs[o2], nout[o2])) return FLR_ERR_ALIAS;
  }
  char* ws = static_cast<char*>(workspace);
  double* sums = reinterpret_cast<double*>(ws + L.sums);
  double* f1 = reinterpret_cast<double*>(ws + L.f1);
  double* s1 = reinterpret_cast<double*>(ws + L.s1);
  double* f2 = reinterpret_cast<double*>(ws + L.f2);
  double* s2 = sums;  // the moment sums are dead once the solve fields exist
  double* red = reinterpret_cast<double*>(ws + L.red);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int H = p->height, W = p->width, r = p->radius;
  // moments: FP64 window sums of the anchored products
  if (flr::launch_box_products(guides, noisy, Q, C, H, W, r, sums, s) != hipSuccess)
    return FLR_ERR_HIP;
  LaunchArgs a = base_args(p);
  a.guides = guides;
  a.noisy = noisy;
  a.gout = grad_out;
  a.sums = sums;
  a.average = p->average_coeffs;
  a.fout = f1;
  if ((st = dispatch(Q, C, flr::K_ADJ_COEF, a, stream)) != FLR_OK) return st;
  // with averaging, s1 = window sums of G / n and g~ G / n (formed from the
  // inputs), then of the coefficients a
  const size_t pl = (size_t)H * W;
  double* s1a = s1 + (size_t)(C + Q * C) * pl;
  if (p->average_coeffs) {
    if (flr::launch_box_avgfields(guides, grad_out, Q, C, H, W, r, s1, s) != hipSuccess ||
        flr::launch_box(f1, s1a, Q * C, H, W, r, s) != hipSuccess)
      return FLR_ERR_HIP;
    a.fin = s1;
  }
  a.fout = f2;
  a.red = red;
  if ((st = dispatch(Q, C, flr::K_ADJ_SOLVE, a, stream)) != FLR_OK) return st;
  if (flr::launch_box(f2, s2, flr::num_sums(Q, C), H, W, r, s) != hipSuccess) return FLR_ERR_HIP;
  a.sums = nullptr;
  a.fin = s2;
  a.fin2 = p->average_coeffs ? s1a : f1;
  a.fout = nullptr;
  a.out = grad_guides;
  a.out2 = grad_noisy;
  if ((st = dispatch(Q, C, flr::K_ADJ_GATHER, a, stream)) != FLR_OK) return st;
  if (grad_reg) {
    const int pblocks = (int)(((size_t)H * W + 255) / 256);
    if (flr::launch_pair_sum(red, pblocks, grad_reg, s) != hipSuccess) return FLR_ERR_HIP;
  }
  return FLR_OK;
}

size_t flr_lowres_workspace_bytes(const flr_params* p, int32_t block, float sigma_low,
                                  int32_t radius_low) {
  if (validate_lowres(p, block, sigma_low, radius_low) != FLR_OK) return 0;
  return lowres_layout(p, block).total;
}

flr_status flr_denoise_lowres(const flr_params* p, int32_t block, float sigma_low,
                              int32_t radius_low, const float* guides, const float* noisy,
                              float* out, void* workspace, size_t workspace_bytes,
                              void* stream) {
  flr_status st = validate_lowres(p, block, sigma_low, radius_low);
  if (st != FLR_OK) return st;
  if ((st = check_ptrs({guides, noisy, out, workspace})) != FLR_OK) return st;
  const LowresLayout L = lowres_layout(p, block);
  if (workspace_bytes < L.total) return FLR_ERR_WORKSPACE;
  const int Q = p->num_guides, C = p->num_channels;
  const size_t pb = plane_bytes(p);
  if (overlaps(out, C * pb, guides, Q * pb) || overlaps(out, C * pb, noisy, C * pb) ||
      overlaps(workspace, L.total, guides, Q * pb) ||
      overlaps(workspace, L.total, noisy, C * pb) || overlaps(workspace, L.total, out, C * pb))
    return FLR_ERR_ALIAS;
  char* ws = static_cast<char*>(workspace);
  double* sums = reinterpret_cast<double*>(ws + L.sums);
  double* tmp = reinterpret_cast<double*>(ws + L.tmp);
  double* coef = reinterpret_cast<double*>(ws + L.coef);
  LaunchArgs a = base_args(p);
  a.guides = guides;
  a.noisy = noisy;
  a.block = block;
  a.Hl = L.Hl;
  a.Wl = L.Wl;
  a.lr_R = radius_low;
  for (int d = -radius_low; d <= radius_low; ++d)
    a.taps[d + radius_low] =
        sigma_low > 0.f ? exp(-(double)(d * d) / (2.0 * (double)sigma_low * (double)sigma_low))
                        : (d == 0 ? 1.0 : 0.0);
  a.fout = sums;
  if ((st = dispatch(Q, C, flr::K_LR_BLOCK, a, stream)) != FLR_OK) return st;
  if (flr::launch_lr_blur(sums, tmp, 1 + flr::num_sums(Q, C), L.Hl, L.Wl, radius_low, a.taps,
                          reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
    return FLR_ERR_HIP;
  a.fin = tmp;
  a.fout = coef;
  if ((st = dispatch(Q, C, flr::K_LR_SOLVE, a, stream)) != FLR_OK) return st;
  a.fin = coef;
  a.fout = nullptr;
  a.out = out;
  a.lr_rows = flr::lr_apply_rows(Q, C, block);
  return dispatch(Q, C, flr::K_LR_APPLY, a, stream);
}

size_t flr_batch_workspace_bytes(const flr_params* p, const flr_frame* frames,
                                 int32_t num_frames) {
  if (validate_batch(p, frames, num_frames) != FLR_OK) return 0;
  return batch_layout(p, frames, num_frames).total;
}

flr_status flr_batch_plan(const flr_params* p, const flr_frame* frames, int32_t n,
                          void* workspace, size_t workspace_bytes, flr_batch* out_plan) {
  flr_status st = validate_batch(p, frames, n);
  if (st != FLR_OK) return st;
  if (!out_plan || !workspace) return FLR_ERR_NULL;
  if (!aligned16(workspace)) return FLR_ERR_ALIGN;
  const BatchLayout L = batch_layout(p, frames, n);
  if (workspace_bytes < L.total) return FLR_ERR_WORKSPACE;
  const int Q = p->num_guides, C = p->num_channels;
  for (int i = 0; i < n; ++i) {
    const flr_frame& f = frames[i];
    const size_t gb = (size_t)Q * f.height * f.width * sizeof(float);
    const size_t nb = (size_t)C * f.noisy_height * f.noisy_width * sizeof(float);
    if (overlaps(workspace, L.total, f.guides, gb) || overlaps(workspace, L.total, f.noisy, nb) ||
        overlaps(workspace, L.total, f.out, (size_t)C * f.height * f.width * sizeof(float)) ||
        (f.guides_low &&
         overlaps(workspace, L.total, f.guides_low,
                  (size_t)Q * f.noisy_height * f.noisy_width * sizeof(float))))
      return FLR_ERR_ALIAS;
  }
  char* ws = static_cast<char*>(workspace);
  LaunchArgs walk[FLR_BATCH_MAX], apply[FLR_BATCH_MAX], up[FLR_BATCH_MAX];
  int ws_walk[FLR_BATCH_MAX + 1], ws_apply[FLR_BATCH_MAX + 1], ws_up[FLR_BATCH_MAX + 1];
  int order[FLR_BATCH_MAX], blocks[FLR_BATCH_MAX];
  flr_params q = *p;
  // the coefficient walk of every plain frame
  int nw = 0;
  for (int i = 0; i < n; ++i) {
    const flr_frame& f = frames[i];
    if (frame_is_joint(f)) continue;
    q.height = f.height;
    q.width = f.width;
    q.tile_rows = f.tile_rows;
    LaunchArgs a = base_args(&q);
    a.guides = f.guides;
    a.noisy = f.noisy;
    a.out = reinterpret_cast<float*>(ws + L.coef[i]);
    a.coef_lo = 1;
    plan(&q, flr::K_COEFFS, &a);
    walk[nw] = a;
    blocks[nw] = a.tiles_x * a.n_seg;
    order[nw] = nw;
    ++nw;
  }
  // largest frames first, so that the small ones fill the tail of the launch
  for (int i = 1; i < nw; ++i)
    for (int j = i; j > 0 && blocks[order[j]] > blocks[order[j - 1]]; --j) {
      const int t = order[j];
      order[j] = order[j - 1];
      order[j - 1] = t;
    }
  LaunchArgs walk_sorted[FLR_BATCH_MAX];
  ws_walk[0] = 0;
  for (int k = 0; k < nw; ++k) {
    walk_sorted[k] = walk[order[k]];
    ws_walk[k + 1] = ws_walk[k] + blocks[order[k]];
  }
  int np = 0, nj = 0;
  ws_apply[0] = ws_up[0] = 0;
  for (int i = 0; i < n; ++i) {
    const flr_frame& f = frames[i];
    q.height = f.height;
    q.width = f.width;
    // as flr_denoise: the segment length of both kernels, unless the frame
    // sets the averaging tiles itself
    q.tile_rows = f.apply_rows > 0 ? f.apply_rows : f.tile_rows;
    LaunchArgs a = base_args(&q);
    a.guides = f.guides;
    a.out = f.out;
    if (!frame_is_joint(f)) {
      a.planes = reinterpret_cast<const float*>(ws + L.coef[i]);
      a.coef_lo = 1;
      plan(&q, flr::K_APPLY_AVG, &a);
      apply[np] = a;
      ws_apply[np + 1] = ws_apply[np] + flr::avg_groups(a.tiles_x * a.n_seg);
      ++np;
    } else {
      a.fin = reinterpret_cast<const double*>(ws + L.mean[i]);
      a.guides_low = f.guides_low;
      a.noisy = f.noisy;
      a.Hl = f.noisy_height;
      a.Wl = f.noisy_width;
      a.up = frame_up(f);
      up[nj] = a;
      ws_up[nj + 1] = ws_up[nj] + (int)(((size_t)f.height * f.width + 255) / 256);
      out_plan->joint_guides[nj] = f.guides_low;
      out_plan->joint_noisy[nj] = f.noisy;
      out_plan->joint_sums[nj] = reinterpret_cast<double*>(ws + L.coef[i]);
      out_plan->joint_models[nj] = reinterpret_cast<double*>(ws + L.models[i]);
      out_plan->joint_mean[nj] = reinterpret_cast<double*>(ws + L.mean[i]);
      out_plan->joint_height[nj] = f.noisy_height;
      out_plan->joint_width[nj] = f.noisy_width;
      ++nj;
    }
  }
  // The persistent launch: one table of launch arguments (the walks, in
  // their sorted order, the averaging, the joint frames' solves and
  // upsampling), the joint frames' box passes, and the stages in queue
  // order: walks, joint sums, joint solves, joint means, averaging, upsampling.
  static thread_local LaunchArgs largs[4 * FLR_BATCH_MAX];
  static thread_local flr::AdjBoxArgs bargs[2 * FLR_BATCH_MAX];
  static thread_local flr::BatchStage stages[4 * FLR_BATCH_MAX];
  int nl = 0, nb = 0, nst = 0, nctr = 0, items = 0;
  int walk_ctr[FLR_BATCH_MAX], inv[FLR_BATCH_MAX];
  auto stage = [&](int kind, int arg, int count, int nx, int wait, int need, int done,
                   int seg_rows, int nseg) {
    stages[nst++] = flr::BatchStage{kind, arg, items, count, nx, wait, need, done, seg_rows,
                                    nseg};
    items += count;
    return count;
  };
  for (int k = 0; k < nw; ++k) {
    const LaunchArgs& a = walk_sorted[k];
    inv[order[k]] = k;
    largs[nl] = a;
    walk_ctr[k] = nctr;
    nctr += a.n_seg;
    stage(flr::BI_WALK, nl++, a.tiles_x * a.n_seg, 0, -1, 0, walk_ctr[k], a.seg_rows, a.n_seg);
  }
  const int fc = (Q + 1) * C;
  int jbox_items[FLR_BATCH_MAX], jsolve_items[FLR_BATCH_MAX], jmean_items[FLR_BATCH_MAX];
  int jctr[FLR_BATCH_MAX], jbox_arg[FLR_BATCH_MAX], jmean_arg[FLR_BATCH_MAX];
  for (int j = 0; j < nj; ++j) {
    flr::AdjBoxArgs b = {};
    b.guides = out_plan->joint_guides[j];
    b.noisy = out_plan->joint_noisy[j];
    b.dst = out_plan->joint_sums[j];
    b.H = out_plan->joint_height[j];
    b.W = out_plan->joint_width[j];
    b.r = p->radius;
    b.Q = Q;
    b.C = C;
    b.count_first = 1;
    // the per-stage run's tiling (same segments: same sums), and the ring
    // where it fits in the persistent kernel's LDS
    const int nx = flr::box_plan(b, 1 + flr::num_sums(Q, C));
    b.ring = flr::box_lds_bytes(b.r, true) <= flr::batch_lds_bytes(Q, C) ? 1 : 0;
    bargs[nb] = b;
    jbox_arg[j] = nb++;
    jctr[j] = nctr;
    nctr += 3;
    jbox_items[j] = stage(flr::BI_JBOX, jbox_arg[j], nx * (1 + flr::num_sums(Q, C)), nx, -1, 0,
                          jctr[j], 0, 0);
  }
  for (int j = 0; j < nj; ++j) {
    LaunchArgs a = base_args(p);
    a.H = a.Hl = out_plan->joint_height[j];
    a.W = a.Wl = out_plan->joint_width[j];
    a.guides = out_plan->joint_guides[j];
    a.fin = out_plan->joint_sums[j];
    a.fout = out_plan->joint_models[j];
    largs[nl] = a;
    jsolve_items[j] = stage(flr::BI_JSOLVE, nl++, (int)(((int64_t)a.H * a.W + 255) / 256), 0,
                            jctr[j], jbox_items[j], jctr[j] + 1, 0, 0);
  }
  for (int j = 0; j < nj; ++j) {
    flr::AdjBoxArgs b = {};
    b.src = out_plan->joint_models[j];
    b.dst = out_plan->joint_mean[j];
    b.count_first = 1;
    b.H = out_plan->joint_height[j];
    b.W = out_plan->joint_width[j];
    b.r = p->radius;
    const int nx = flr::box_plan(b, fc);
    b.ring = flr::box_lds_bytes(b.r, true) <= flr::batch_lds_bytes(Q, C) ? 1 : 0;
    bargs[nb] = b;
    jmean_arg[j] = nb++;
    jmean_items[j] = stage(flr::BI_JMEAN, jmean_arg[j], nx * fc, nx, jctr[j] + 1,
                           jsolve_items[j], jctr[j] + 2, 0, 0);
  }
  for (int i = 0; i < np; ++i) {
    const LaunchArgs& a = apply[i];
    const LaunchArgs& w = walk_sorted[inv[i]];
    largs[nl] = a;
    stage(flr::BI_AVG, nl++, a.tiles_x * a.n_seg, 0, walk_ctr[inv[i]], w.tiles_x, -1,
          w.seg_rows, w.n_seg);
  }
  for (int j = 0; j < nj; ++j) {
    const LaunchArgs& a = up[j];
    largs[nl] = a;
    stage(flr::BI_UP, nl++, (int)(((int64_t)a.H * a.W + 255) / 256), 0, jctr[j] + 2,
          jmean_items[j], -1, 0, 0);
  }
  flr::BatchPlanDev pd = {};
  pd.stages = reinterpret_cast<const flr::BatchStage*>(ws + L.stages);
  pd.nstages = nst;
  pd.nitems = items;
  pd.ncounters = nctr;
  pd.largs = reinterpret_cast<const LaunchArgs*>(ws + L.largs);
  pd.bargs = reinterpret_cast<const flr::AdjBoxArgs*>(ws + L.bargs);
  pd.ctl = reinterpret_cast<int*>(ws + L.ctl);
  pd.counters = reinterpret_cast<int*>(ws + L.counters);
  if ((size_t)nctr > L.ncounters) return FLR_ERR_WORKSPACE;  // never: the layout's bound
  if (hipMemcpy(ws + L.largs, largs, nl * sizeof(LaunchArgs), hipMemcpyHostToDevice) !=
          hipSuccess ||
      (nb && hipMemcpy(ws + L.bargs, bargs, nb * sizeof(flr::AdjBoxArgs),
                       hipMemcpyHostToDevice) != hipSuccess) ||
      hipMemcpy(ws + L.stages, stages, nst * sizeof(flr::BatchStage), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(ws + L.pdev, &pd, sizeof pd, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(ws + L.ctl, 0, 4 * sizeof(int)) != hipSuccess ||
      hipMemset(ws + L.counters, 0, L.ncounters * sizeof(int)) != hipSuccess)
    return FLR_ERR_HIP;
  out_plan->num_items = items;
  out_plan->persistent_blocks = items < flr::kCUs ? items : flr::kCUs;
  out_plan->persistent_plan = ws + L.pdev;

  // tables of the per-stage launches: launch arguments, then the three
  // workgroup offset arrays
  int starts[3 * (FLR_BATCH_MAX + 1)];
  for (int k = 0; k <= n; ++k) {
    starts[k] = k <= nw ? ws_walk[k] : 0;
    starts[(n + 1) + k] = k <= np ? ws_apply[k] : 0;
    starts[2 * (n + 1) + k] = k <= nj ? ws_up[k] : 0;
  }
  if ((nw && hipMemcpy(ws + L.walk, walk_sorted, nw * sizeof(LaunchArgs),
                       hipMemcpyHostToDevice) != hipSuccess) ||
      (np && hipMemcpy(ws + L.apply, apply, np * sizeof(LaunchArgs), hipMemcpyHostToDevice) !=
                 hipSuccess) ||
      (nj && hipMemcpy(ws + L.up, up, nj * sizeof(LaunchArgs), hipMemcpyHostToDevice) !=
                 hipSuccess) ||
      hipMemcpy(ws + L.starts, starts, 3 * (n + 1) * sizeof(int), hipMemcpyHostToDevice) !=
          hipSuccess)
    return FLR_ERR_HIP;
  out_plan->params = *p;
  out_plan->num_frames = n;
  out_plan->num_joint = nj;
  out_plan->coeff_blocks = ws_walk[nw];
  out_plan->apply_blocks = ws_apply[np];
  out_plan->up_blocks = ws_up[nj];
  out_plan->walk_table = ws + L.walk;
  out_plan->apply_table = ws + L.apply;
  out_plan->up_table = ws + L.up;
  out_plan->walk_starts = reinterpret_cast<int*>(ws + L.starts);
  return FLR_OK;
}

flr_status flr_batch_failed(const flr_batch* b, int32_t* failed) {
  if (!b || !failed || !b->persistent_plan) return FLR_ERR_NULL;
  flr::BatchPlanDev pd;
  int flag = 0;
  if (hipMemcpy(&pd, b->persistent_plan, sizeof pd, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&flag, pd.ctl + 2, sizeof flag, hipMemcpyDeviceToHost) != hipSuccess)
    return FLR_ERR_HIP;
  *failed = flag != 0;
  return FLR_OK;
}

flr_status flr_batch_run(const flr_batch* b, void* stream) {
  if (!b || !b->walk_table) return FLR_ERR_NULL;
  const flr_params* p = &b->params;
  const int Q = p->num_guides, C = p->num_channels, n = b->num_frames;
  const int np = n - b->num_joint, nj = b->num_joint;
  const int* starts = b->walk_starts;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  flr_status st;
  LaunchArgs a = base_args(p);
  if (b->persistent_blocks < 0) return FLR_ERR_MODE;
  if (b->persistent_blocks > 0) {
    if (!b->persistent_plan) return FLR_ERR_NULL;
    a.bplan = static_cast<const flr::BatchPlanDev*>(b->persistent_plan);
    a.batch_blocks = b->persistent_blocks;
    return dispatch(Q, C, flr::K_BATCH_PERSISTENT, a, stream);
  }
  if (np > 0) {
    a.frames = static_cast<const LaunchArgs*>(b->walk_table);
    a.wg_start = starts;
    a.nframes = np;
    a.batch_blocks = b->coeff_blocks;
    if ((st = dispatch(Q, C, flr::K_COEFFS_BATCH, a, stream)) != FLR_OK) return st;
    a.frames = static_cast<const LaunchArgs*>(b->apply_table);
    a.wg_start = starts + (n + 1);
    a.batch_blocks = b->apply_blocks;
    if ((st = dispatch(Q, C, flr::K_APPLY_AVG_BATCH, a, stream)) != FLR_OK) return st;
  }
  if (nj > 0) {
    for (int k = 0; k < nj; ++k) {
      const int h = b->joint_height[k], w = b->joint_width[k];
      if (flr::launch_box_products(b->joint_guides[k], b->joint_noisy[k], Q, C, h, w, p->radius,
                                   b->joint_sums[k], s, true) != hipSuccess)
        return FLR_ERR_HIP;
      LaunchArgs j = base_args(p);
      j.H = j.Hl = h;
      j.W = j.Wl = w;
      j.guides = b->joint_guides[k];
      j.fin = b->joint_sums[k];
      j.fout = b->joint_models[k];
      if ((st = dispatch(Q, C, flr::K_LR_SOLVE, j, stream)) != FLR_OK) return st;
      if (flr::launch_mean_planes64(b->joint_models[k], b->joint_mean[k], (Q + 1) * C, h, w,
                                    p->radius, s) != hipSuccess)
        return FLR_ERR_HIP;
    }
    a.frames = static_cast<const LaunchArgs*>(b->up_table);
    a.wg_start = starts + 2 * (n + 1);
    a.nframes = nj;
    a.batch_blocks = b->up_blocks;
    if ((st = dispatch(Q, C, flr::K_UP_APPLY_BATCH, a, stream)) != FLR_OK) return st;
  }
  return FLR_OK;
}

const char* flr_status_str(flr_status s) {
  switch (s) {
    case FLR_OK: return "ok";
    case FLR_ERR_NULL: return "null pointer argument";
    case FLR_ERR_SHAPE: return "height/width out of range";
    case FLR_ERR_RADIUS: return "radius out of range";
    case FLR_ERR_EPS: return "eps/eps_mul negative or not finite";
    case FLR_ERR_CHANNELS: return "number of guides or channels out of range";
    case FLR_ERR_ALIAS: return "output overlaps an input";
    case FLR_ERR_ALIGN: return "pointer not 16-byte aligned";
    case FLR_ERR_WORKSPACE: return "workspace missing or too small";
    case FLR_ERR_MODE: return "invalid reg_mode, flags or boolean field";
    case FLR_ERR_HIP: return "HIP launch failed";
  }
  return "unknown status";
}

}  // extern "C"
