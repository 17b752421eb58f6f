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
size_t unfused_coeff_offset(const flr_params* p) {
  const size_t mb = flr_num_moment_planes(p->num_guides, p->num_channels) * plane_bytes(p);
  return (mb + 255) / 256 * 256;
}

// Workspace of flr_denoise_backward, byte offsets of 256-aligned FP64
// regions: the window sums of the anchored input products (later reused for
// the window sums of the solve fields), the averaging fields, their window
// sums (with averaging only), the solve fields, and the per-workgroup sums
// of the regulariser gradients.
struct BackwardLayout {
  size_t sums, f1, s1, f2, red, total;
};

BackwardLayout backward_layout(const flr_params* p) {
  const int Q = p->num_guides, C = p->num_channels;
  const size_t pl = (size_t)p->height * p->width;
  const size_t pblocks = (pl + 255) / 256;
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t ns = (size_t)flr::num_sums(Q, C), nf1 = (size_t)flr::num_avg_fields(Q, C);
  BackwardLayout L{};
  size_t o = 0;
  L.sums = o;
  o += al(ns * pl * sizeof(double));
  L.f1 = o;
  o += al(nf1 * pl * sizeof(double));
  L.s1 = o;
  if (p->average_coeffs) o += al(nf1 * pl * sizeof(double));
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
  if (p->flags & ~(uint32_t)FLR_FLAG_RAW_MOMENTS) return FLR_ERR_MODE;
  if (p->tile_rows < 0) return FLR_ERR_SHAPE;
  return FLR_OK;
}

size_t flr_denoise_workspace_bytes(const flr_params* p) {
  if (flr_validate_params(p) != FLR_OK) return 0;
  const size_t pb = plane_bytes(p);
  if (p->fused == FLR_PATH_STAGES)
    return unfused_coeff_offset(p) + flr_num_coeff_planes(p->num_guides, p->num_channels) * pb;
  if (!p->average_coeffs) return 0;
  if (p->fused == FLR_PATH_TWO_PASS && !flr::split_walk(p->num_guides, p->num_channels))
    return flr_num_coeff_planes(p->num_guides, p->num_channels) * pb;
  if (p->fused == FLR_PATH_TWO_PASS)  // split walks take the stage sequence
    return unfused_coeff_offset(p) + flr_num_coeff_planes(p->num_guides, p->num_channels) * pb;
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
  const size_t cb = flr_num_coeff_planes(p->num_guides, p->num_channels) * pb;
  if (overlaps(coeffs, cb, guides, p->num_guides * pb) ||
      overlaps(coeffs, cb, noisy, p->num_channels * pb))
    return FLR_ERR_ALIAS;
  LaunchArgs a = base_args(p);
  a.guides = guides;
  a.noisy = noisy;
  a.out = coeffs;
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
      overlaps(out, ob, coeffs, flr_num_coeff_planes(p->num_guides, p->num_channels) * pb))
    return FLR_ERR_ALIAS;
  LaunchArgs a = base_args(p);
  a.guides = guides;
  a.planes = coeffs;
  a.out = out;
  const int kind = p->average_coeffs ? flr::K_APPLY_AVG : flr::K_APPLY_POINT;
  if (kind == flr::K_APPLY_AVG) plan(p, kind, &a);
  return dispatch(p->num_guides, p->num_channels, kind, a, stream);
}

flr_status flr_denoise(const flr_params* p, const float* guides, const float* noisy, float* out,
                       void* workspace, size_t workspace_bytes, void* stream) {
  flr_status st = flr_validate_params(p);
  if (st != FLR_OK) return st;
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
  if (p->fused == FLR_PATH_TWO_PASS && p->average_coeffs && !flr::split_walk(Q, C)) {
    float* coeffs = static_cast<float*>(workspace);
    if ((st = flr_coefficients(p, guides, noisy, coeffs, stream)) != FLR_OK) return st;
    return flr_apply(p, guides, coeffs, out, stream);
  }
  // Too many moment channels for one LDS-resident walk: the two-pass path
  // takes the stage sequence, whose moment walk is split into two slices.
  const bool stages = p->fused == FLR_PATH_STAGES ||
                      (p->fused == FLR_PATH_TWO_PASS && p->average_coeffs);
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
  if (p->average_coeffs) {
    if (flr::launch_box(f1, s1, flr::num_avg_fields(Q, C), H, W, r, s) != hipSuccess)
      return FLR_ERR_HIP;
    a.fin = s1;
  }
  a.fout = f2;
  a.red = red;
  if ((st = dispatch(Q, C, flr::K_ADJ_SOLVE, a, stream)) != FLR_OK) return st;
  if (flr::launch_box(f2, s2, flr::num_sums(Q, C), H, W, r, s) != hipSuccess) return FLR_ERR_HIP;
  a.sums = nullptr;
  a.fin = s2;
  a.fin2 = p->average_coeffs ? s1 : f1;
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
