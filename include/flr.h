/*
 * flr.h - C ABI of the Fast Local Regression (FLR) library for AMD MI355X (gfx950).
 *
 * FLR fits, for every pixel k, a regularised affine model from a set of
 * noise-free guide images to a noisy image over the square window T_k of
 * radius r centred on k, and evaluates it at k (Sec. 3.1, Eqs. matX, matY,
 * closed_form; Sec. 3.2). The window is clipped to the image, so it holds
 * n_k = (rows of T_k inside the image) x (columns inside) pixels.
 *
 * The path has four stages, each with its own entry point, plus a fused one:
 *   flr_moments  window moments of the guides and the noisy image (Sec. 3.2:
 *                box-filtering the outer-product tensors gives X_k^T X_k and
 *                X_k^T Y_k exactly), returned as central moments;
 *   flr_solve    the regularised small SPD solve per pixel (Eq. closed_form
 *                with Eq. tikhonov, or the Appendix normalisation);
 *   flr_coefficients  the two above in one pass, without the moment image;
 *   flr_apply    optional window-average of the coefficients, then the
 *                reconstruction I_k = x_k A_k (Sec. 3.1);
 *   flr_denoise  all of the above: in one fused kernel, in two kernels
 *                (moments + solve, then average + reconstruction), or as the
 *                three stage entry points (see flr_path);
 *   flr_denoise_backward  its adjoint: gradients with respect to the guides,
 *                the noisy image and the regularisers;
 *   flr_denoise_lowres  the paper's fast variant: block-downsampled moments,
 *                a low-resolution Gaussian blur and solve, bilinearly
 *                interpolated models.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Arrays are planar float32, each plane dense row-major [H][W] with the
 * planes back to back (plane stride H*W elements):
 *   guides  [Q][H][W]   the Q guide images, WITHOUT the constant-1 guide,
 *                       which is always implied (Sec. 3.1: the first column
 *                       of X_k is all ones);
 *   noisy   [C][H][W]   the noisy channels (Y);
 *   out     [C][H][W]   the reconstruction;
 *   moments [M][H][W]   M = flr_num_moment_planes(Q, C) planes, in order
 *                       n | mu_g[Q] | nu_y[C] | Wcov upper triangle row-major
 *                       [Q(Q+1)/2] | Vcov[q][c] row-major [Q*C], where mu, nu
 *                       are window means, Wcov = S/n - mu mu^T (the
 *                       Appendix's W) and Vcov = X^T Y / n - mu nu^T;
 *   coeffs  [F*C][H][W] F = Q+1 planes per channel, in order b[c] for every
 *                       c, then a[q][c] row-major: the model at pixel k is
 *                       y_c = b[c] + sum_q g_q a[q][c] in original units.
 *
 * Regulariser (eps is added in covariance scale, i.e. to moments divided by
 * n, so its meaning does not depend on the window size):
 *   FLR_REG_RIDGE  (Wcov + eps I) a = Vcov, b = nu - a^T mu: Eq. tikhonov
 *                  with the bias coefficient left unpenalised;
 *   FLR_REG_PAPER  the Appendix normalisation: W^ = Wcov + eps_mul (mu mu^T +
 *                  diag(mu o mu)) + eps I, then the correlation-matrix solve
 *                  (C^ + eps I) A^ = B^, which equals
 *                  (W^ + eps diag(W^)) a = Vcov.
 *
 * Ownership: every pointer is caller-owned DEVICE memory (e.g. the data
 * pointer of a torch tensor on the current GPU); the library never
 * allocates, keeps no per-call state and is reentrant. `stream` is a
 * hipStream_t (NULL = the default stream). Pointers must be 16-byte aligned.
 * Outputs may not overlap inputs.
 *
 * Errors: arguments are validated on the host before any HIP call; a
 * non-zero flr_status is returned and nothing is launched. A launch failure
 * returns FLR_ERR_HIP. Kernels run asynchronously on `stream`; faults
 * surface at the caller's next synchronisation. NaN/Inf inputs propagate to
 * the outputs; nothing is clamped except Cholesky pivots, which are kept
 * >= 1e-30 so that a singular system (eps = 0, flat window) stays finite.
 */
#ifndef FLR_H
#define FLR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FLR_MAX_GUIDES 12   /* Q: 1..12 guides, plus the implied constant */
#define FLR_MAX_CHANNELS 4  /* C: 1..4 noisy channels */
#define FLR_MAX_RADIUS 32   /* r: 0..32, window (2r+1)^2 */
#define FLR_MAX_DIM 32768   /* H, W: 1..32768 */

typedef enum {
  FLR_OK = 0,
  FLR_ERR_NULL = 1,       /* a required pointer is NULL */
  FLR_ERR_SHAPE = 2,      /* height/width outside 1..FLR_MAX_DIM */
  FLR_ERR_RADIUS = 3,     /* radius outside 0..FLR_MAX_RADIUS */
  FLR_ERR_EPS = 4,        /* eps or eps_mul negative or not finite */
  FLR_ERR_CHANNELS = 5,   /* num_guides or num_channels out of range */
  FLR_ERR_ALIAS = 6,      /* an output overlaps an input */
  FLR_ERR_ALIGN = 7,      /* a pointer is not 16-byte aligned */
  FLR_ERR_WORKSPACE = 8,  /* workspace missing or smaller than required */
  FLR_ERR_MODE = 9,       /* reg_mode / fused / flags / boolean field invalid */
  FLR_ERR_HIP = 10        /* a HIP launch failed */
} flr_status;

typedef enum { FLR_REG_RIDGE = 0, FLR_REG_PAPER = 1 } flr_reg_mode;

/* flr_denoise execution paths (flr_params.fused) */
typedef enum {
  FLR_PATH_STAGES = 0,   /* flr_moments -> flr_solve -> flr_apply, images in the workspace */
  FLR_PATH_FUSED = 1,    /* one kernel: moments, solve, average, reconstruction; with
                            averaging, coefficients pass through a per-workgroup ring
                            in the workspace and r coefficient rows are recomputed at
                            each workgroup's top and bottom */
  FLR_PATH_TWO_PASS = 2  /* with averaging: one kernel for moments and solve writing the
                            coefficient image to the workspace, then the averaging and
                            reconstruction of flr_apply; the image holds each intercept
                            as an FP32 pair (hi, lo: (Q + 2) * C planes), formed in FP64
                            from the slopes as stored (FLR_FLAG_INTERCEPT_PAIR's
                            layout, always); without averaging: as FUSED */
} flr_path;

/* flags */
#define FLR_FLAG_RAW_MOMENTS 1u /* flr_moments only: write raw window sums
                                   n | sum g | sum y | sum g_p g_q | sum g_q y_c
                                   (same plane order, nothing centred or divided).
                                   Exact for small-integer inputs. */
#define FLR_FLAG_INTERCEPT_PAIR 2u /* flr_coefficients writes, flr_apply reads, a
                                   coefficient image of (Q + 2) * C planes: b (hi) [C],
                                   a [Q][C], b (lo) [C]. The intercept is formed in
                                   FP64 from the slopes as stored (FP32) and kept as
                                   hi + lo, so that windows whose intercept and slope
                                   terms cancel (nearly collinear guides) keep FP64
                                   accuracy in the output where one FP32 intercept
                                   does not. flr_solve, flr_denoise_backward,
                                   flr_denoise_lowres and the batch calls reject it
                                   (FLR_ERR_MODE); flr_moments, flr_denoise and
                                   flr_flnr_denoise ignore it. */

typedef struct {
  int32_t height, width;   /* H, W in pixels */
  int32_t num_guides;      /* Q, excluding the implied constant guide */
  int32_t num_channels;    /* C */
  int32_t radius;          /* r */
  float eps;               /* additive regulariser, finite, >= 0 */
  float eps_mul;           /* FLR_REG_PAPER multiplicative term, finite, >= 0 */
  int32_t reg_mode;        /* flr_reg_mode */
  int32_t average_coeffs;  /* 1: average (b, a) over the window before
                              reconstruction; 0: use the pixel's own model */
  int32_t fused;           /* flr_denoise: an flr_path */
  uint32_t flags;          /* FLR_FLAG_* */
  int32_t tile_rows;       /* rows per workgroup segment; 0 = automatic */
  const float* eps_device; /* optional: device float[2] holding (eps, eps_mul), read by the
                              kernels when they run in place of the two fields above, so
                              that a training loop can update the regularisers on the
                              device (flr_reg_adam_step, flr_train.h) without a host read;
                              the values must stay finite and >= 0 (not checked). NULL:
                              eps and eps_mul above. 4-byte aligned. */
} flr_params;

/* Number of moment planes M = 1 + Q + C + Q(Q+1)/2 + Q*C (0 if out of range). */
size_t flr_num_moment_planes(int32_t num_guides, int32_t num_channels);
/* Number of coefficient planes (Q+1)*C (0 if out of range). */
size_t flr_num_coeff_planes(int32_t num_guides, int32_t num_channels);

/* Workspace bytes flr_denoise needs for these parameters (0 if invalid):
 * FLR_PATH_STAGES: the moment and coefficient images, (M + F*C)*H*W floats
 * (the coefficient image starts at the next 256-byte boundary);
 * FLR_PATH_FUSED with averaging: a per-workgroup ring of 2r+1 coefficient rows;
 * FLR_PATH_TWO_PASS with averaging: the coefficient image with intercept
 * pairs, (F + 1)*C*H*W floats (F = Q + 1; when Q + C + Q(Q+1)/2 + Q*C
 * exceeds 78 moment channels the walk is split in two: first a moment
 * image of M planes, of which the first slice's are written, then the
 * coefficient image at the next 256-byte boundary);
 * without averaging: 0 (STAGES aside). Depends on the launch geometry only. */
size_t flr_denoise_workspace_bytes(const flr_params* p);

/* Window moments (Sec. 3.2). Reads guides, noisy; writes moments [M][H][W]. */
flr_status flr_moments(const flr_params* p, const float* guides, const float* noisy,
                       float* moments, void* stream);

/* Per-pixel regularised solve (Eq. closed_form with Eq. tikhonov / Appendix).
 * Reads central moments [M][H][W] as written by flr_moments; writes coeffs
 * [F*C][H][W] in original units. Uses reg_mode, eps, eps_mul. */
flr_status flr_solve(const flr_params* p, const float* moments, float* coeffs, void* stream);

/* Moments and solve in one pass (no moment image): writes the coefficient
 * planes [F*C][H][W] in original units, the result of flr_moments followed
 * by flr_solve, with the window sums and the solve kept in FP64/FP32 on chip.
 * Uses radius, reg_mode, eps, eps_mul, tile_rows. */
flr_status flr_coefficients(const flr_params* p, const float* guides, const float* noisy,
                            float* coeffs, void* stream);

/* Window-average of the coefficients if p->average_coeffs (same clipped
 * window as the moments), then reconstruction out_c = b_c + sum_q g_q a_qc
 * (Sec. 3.1). Reads guides and coeffs; writes out [C][H][W]. */
flr_status flr_apply(const flr_params* p, const float* guides, const float* coeffs,
                     float* out, void* stream);

/* The whole path. workspace must hold flr_denoise_workspace_bytes(p) bytes
 * (NULL allowed when that is 0). Concurrent calls must use distinct
 * workspaces. */
flr_status flr_denoise(const flr_params* p, const float* guides, const float* noisy,
                       float* out, void* workspace, size_t workspace_bytes, void* stream);

/* Workspace bytes of flr_denoise_backward (0 if invalid): FP64 images of
 * the window moments, the coefficients, the adjoint's per-pixel fields and,
 * with averaging, the window sums of the averaging fields, about
 * (2*(M - 1) + Q*C + (C + 2*Q*C if averaging))*8 bytes per pixel. */
size_t flr_denoise_backward_workspace_bytes(const flr_params* p);

/* Gradients of flr_denoise (its adjoint; Sec. 3.3 trains the guide network
 * through FLR, the Appendix learns eps and eps_mul by backpropagation). For a
 * loss L with grad_out = dL/d(out) [C][H][W], out = flr_denoise(p, guides,
 * noisy), writes grad_guides = dL/d(guides) [Q][H][W] and grad_noisy =
 * dL/d(noisy) [C][H][W] (FP32) and, unless grad_reg is NULL, grad_reg[0] =
 * dL/d(eps) and grad_reg[1] = dL/d(eps_mul) (device FP64; the latter is 0
 * in ridge mode). The moments and coefficients are recomputed from guides
 * and noisy, in FP64; nothing of the forward call is needed. Where the forward
 * clamped a guide's rounded-negative window variance to 0, no gradient
 * flows through that variance. p->fused is ignored; p->flags must be 0.
 * workspace must hold flr_denoise_backward_workspace_bytes(p) bytes.
 * Errors as flr_denoise, and FLR_ERR_ALIAS when an output overlaps an
 * input, another output or the workspace. */
flr_status flr_denoise_backward(const flr_params* p, const float* guides, const float* noisy,
                                const float* grad_out, float* grad_guides, float* grad_noisy,
                                double* grad_reg, void* workspace, size_t workspace_bytes,
                                void* stream);

/* The paper's fast variant (Sec. 3.2, its four-stage implementation): the
 * outer-product moments summed over block x block pixel blocks (a strided
 * box filter), a Gaussian blur of the low-resolution moment planes with
 * weights exp(-d^2 / (2 sigma_low^2)) for |d| <= radius_low along each axis
 * (zero outside the low-resolution grid; sigma_low = 0 keeps the block
 * alone), one regularised solve per low-resolution pixel (reg_mode, eps,
 * eps_mul in covariance scale, as flr_solve), and the models interpolated
 * bilinearly at every full-resolution pixel (low-resolution coordinate
 * (i + 0.5) / block - 0.5, clamped to the grid) and applied there:
 * out_c = b_c + sum_q g_q a_qc. The last block row/column is ragged when
 * the size is not a multiple of block. p->radius, p->average_coeffs and
 * p->fused are not used; p->flags must be 0. block: 1, 2, 4, 8 or 16
 * (else FLR_ERR_MODE); sigma_low finite and >= 0 (else FLR_ERR_EPS);
 * radius_low 0..8 (else FLR_ERR_RADIUS). Workspace: FP64 low-resolution
 * planes, flr_lowres_workspace_bytes(). Other errors as flr_denoise. */
size_t flr_lowres_workspace_bytes(const flr_params* p, int32_t block, float sigma_low,
                                  int32_t radius_low);
flr_status flr_denoise_lowres(const flr_params* p, int32_t block, float sigma_low,
                              int32_t radius_low, const float* guides, const float* noisy,
                              float* out, void* workspace, size_t workspace_bytes,
                              void* stream);

/* Batched serving (Sec. 3.2 measures whole frames; joint denoising and
 * upsampling, Sec. 3.2, is one of the frame kinds): frames of uneven size
 * through the two-pass path with coefficient averaging, each stage one
 * launch over the tiles of every frame. A plain frame has its noisy input
 * on the output grid. A joint frame has it on a grid `up` times coarser in
 * each direction (up = 2, 4 or 8, height = up * noisy_height, width =
 * up * noisy_width) together with guides rasterised on that grid
 * (guides_low): its coefficients are fitted and window-averaged there (in
 * FP64: the models are then applied to guides the fit did not see, which
 * exposes the error an FP32 factorisation leaves in them), interpolated
 * bilinearly (half-pixel centres, clamped) at every output pixel and
 * applied to the full-resolution guides. */
#define FLR_BATCH_MAX 64

typedef struct {
  int32_t height, width;              /* output grid, and the guides' */
  int32_t noisy_height, noisy_width;  /* the noisy input's grid */
  int32_t tile_rows;                  /* rows per workgroup of the coefficient walk; 0 = planned */
  int32_t apply_rows;                 /* rows per workgroup of the averaging (at most 17); 0 =
                                         as tile_rows (flr_denoise's choice: same tiles, same
                                         results bit for bit) */
  const float* guides;                /* [Q][height][width] */
  const float* guides_low;            /* joint frames: [Q][noisy_height][noisy_width]; else NULL */
  const float* noisy;                 /* [C][noisy_height][noisy_width] */
  float* out;                         /* [C][height][width] */
} flr_frame;

/* Launch plan of a batch, filled by flr_batch_plan and only read by
 * flr_batch_run. It points into the plan's workspace, which must stay
 * allocated and untouched while the plan is used. */
typedef struct {
  flr_params params;
  int32_t num_frames, num_joint;
  int32_t coeff_blocks, apply_blocks, up_blocks;
  int32_t persistent_blocks;          /* workgroups of the persistent launch (the plan sets
                                         one per compute unit, at most num_items); 0 runs
                                         one launch per stage instead. The caller may
                                         change it between flr_batch_plan and flr_batch_run. */
  int32_t num_items;                  /* work items of the persistent launch */
  void* walk_table;                   /* device: per-frame launch arguments of the walk */
  void* apply_table;                  /* device: ... of the averaging kernel (plain frames) */
  void* up_table;                     /* device: ... of the upsampling kernel (joint frames) */
  int* walk_starts;                   /* device: workgroup offsets of the per-stage launches */
  void* persistent_plan;              /* device: the persistent launch's stage table, launch
                                         arguments, queue head and completion counters */
  /* joint frames, fitted on the noisy grid in FP64 */
  const float* joint_guides[FLR_BATCH_MAX]; /* the frame's guides_low */
  const float* joint_noisy[FLR_BATCH_MAX];  /* the frame's noisy input */
  double* joint_sums[FLR_BATCH_MAX];        /* device: window count and moment sums */
  double* joint_models[FLR_BATCH_MAX];      /* device: the fitted models */
  double* joint_mean[FLR_BATCH_MAX];        /* device: ... window-averaged */
  int32_t joint_height[FLR_BATCH_MAX], joint_width[FLR_BATCH_MAX];
} flr_batch;

/* Workspace bytes of a batch (0 if invalid): the launch tables, the
 * coefficient image (FP32, intercept pairs) of every plain frame, and for every joint frame
 * FP64 images on its noisy grid: the window count and moment sums, the
 * models and their window means. */
size_t flr_batch_workspace_bytes(const flr_params* p, const flr_frame* frames,
                                 int32_t num_frames);

/* Validates the batch (p: num_guides, num_channels, radius, eps, eps_mul,
 * reg_mode; average_coeffs must be 1, flags 0; every frame as flr_denoise
 * would check it; at most FLR_BATCH_MAX frames; the walk must fit one pass,
 * Q + C + Q(Q+1)/2 + Q*C <= 78, else FLR_ERR_CHANNELS), plans every frame's
 * tiles (tile_rows, or the planned segment length), orders the walk's
 * frames largest first, and copies the launch tables into the workspace
 * (a synchronous copy: not for graph capture). */
flr_status flr_batch_plan(const flr_params* p, const flr_frame* frames, int32_t num_frames,
                          void* workspace, size_t workspace_bytes, flr_batch* plan);

/* Runs a planned batch on `stream`. With plan->persistent_blocks > 0 (the
 * default) it is ONE launch of that many persistent workgroups, which take
 * work items in order from a device queue: the coefficient walk's tiles of
 * every plain frame (largest frames first); per joint frame the tiles of
 * its FP64 window sums, its per-pixel solve and the window mean of its
 * models; the averaging and reconstruction tiles of the plain frames; the
 * upsampling of the joint frames. An item waits (on device counters) only
 * for the items it reads, all of which come earlier in the queue; a
 * workgroup always finishes its item before taking the next, so every wait
 * ends. The last workgroup to finish resets the queue and the counters, so
 * the launch can be captured in a HIP graph and replayed (runs of one plan
 * must not overlap). With persistent_blocks = 0: one launch per stage (the
 * walk over all plain frames, their averaging, per joint frame its three
 * FP64 stages, the upsampling). Kernel launches only, in both cases. */
flr_status flr_batch_run(const flr_batch* plan, void* stream);

/* Whether a persistent run of this plan gave up waiting for an item's
 * inputs (a wait longer than about a second, which a correct run never
 * has): *failed = 1 (kept until the plan is made again), else 0. A
 * synchronous read of a device flag: call after the runs have completed.
 * FLR_ERR_NULL for null pointers, FLR_ERR_HIP if the read fails. */
flr_status flr_batch_failed(const flr_batch* plan, int32_t* failed);

/* Static description of a status code. */
const char* flr_status_str(flr_status s);

/* Host-only argument check used by every entry point (no HIP call). */
flr_status flr_validate_params(const flr_params* p);

#ifdef __cplusplus
}
#endif

#endif /* FLR_H */
