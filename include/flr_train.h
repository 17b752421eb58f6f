/*
 * flr_train.h - C ABI of the element-wise stages of an FLNR training step.
 *
 * Sec. 3.3 trains the guide network end to end: the denoised output's loss
 * is backpropagated through the regression (flr_denoise_backward, flr.h) and
 * the network (flr_net_backward, flr_net.h) into the weights. A step on a
 * batch of crops is, per crop, flr_net_forward -> flr_denoise over the 12
 * guides -> flr_l1_loss_grad -> flr_denoise_backward -> flr_net_backward
 * (accumulating), and then one flr_adamw_step on the FP32 master weights.
 *
 * Ownership and errors as in flr.h: caller-owned device memory, 16-byte
 * aligned; nothing is allocated; arguments are checked on the host before
 * any launch; FLR_ERR_HIP on launch failure. Kernels run on `stream`.
 */
#ifndef FLR_TRAIN_H
#define FLR_TRAIN_H

#include <stddef.h>
#include <stdint.h>

#include "flr.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Workspace bytes of flr_l1_loss_grad for n values (0 when n is outside
 * 1..2^34). */
size_t flr_l1_workspace_bytes(int64_t n);

/* L1 loss and its gradient over n FP32 values: *loss = scale * sum |out[i] -
 * target[i]| (FP64, summed in a fixed order), grad[i] = scale * sign(out[i] -
 * target[i]) with sign(0) = 0 (the difference taken in FP32). scale = 1 /
 * (number of values in the batch) gives the mean absolute error. loss is one
 * device double (8-byte alignment suffices, so a batch's losses can sit side
 * by side in one array). FLR_ERR_SHAPE for n outside 1..2^34, FLR_ERR_EPS for a scale
 * that is not finite, FLR_ERR_ALIAS when an output overlaps an input or
 * another output. */
flr_status flr_l1_loss_grad(int64_t n, const float* out, const float* target, float scale,
                            float* grad, double* loss, void* workspace, size_t workspace_bytes,
                            void* stream);

/* flr_l1_loss_grad for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving or training loops, harnesses that
 * forbid allocation): the same kernels and the same fixed-order sums, so the
 * results equal flr_l1_loss_grad's bit for bit, with the per-workgroup
 * partial sums in a scratch array the library holds on each GPU for the
 * life of the process (1024 doubles, 8 KiB; enough for every n up to 2^34,
 * larger n is FLR_ERR_SHAPE). The call allocates nothing. Every call on one
 * GPU shares that GPU's array: calls that may overlap on one GPU (on
 * different streams without ordering) race and must not be issued. The
 * array's device address is looked up on the first call made with each
 * device current (FLR_ERR_HIP if that fails). Other errors as
 * flr_l1_loss_grad. */
flr_status flr_l1_loss_grad_noalloc(int64_t n, const float* out, const float* target,
                                    float scale, float* grad, double* loss, void* stream);

/* One AdamW step (Adam with decoupled weight decay) on n FP32 parameters, in
 * place: with t = step (1 for the first update),
 *   p <- p - lr * weight_decay * p
 *   m <- beta1 m + (1 - beta1) g,   v <- beta2 v + (1 - beta2) g^2
 *   p <- p - lr / (1 - beta1^t) * m / (sqrt(v) / sqrt(1 - beta2^t) + eps)
 * m and v (zero before the first step) are updated in place. FP32
 * arithmetic; the bias corrections are formed in FP64 on the host.
 * FLR_ERR_MODE for step < 1, FLR_ERR_EPS for a negative or non-finite
 * hyperparameter or beta >= 1, FLR_ERR_ALIAS when two of the arrays overlap. */
flr_status flr_adamw_step(int64_t n, float* params, const float* grads, float* m, float* v,
                          int32_t step, float lr, float beta1, float beta2, float eps,
                          float weight_decay, void* stream);

/* Adam on the logarithms of FLR's regularisers, on the device (the
 * Appendix learns its regularisers by backpropagation; the logarithm keeps
 * them positive): reg = device float[2] (eps, eps_mul), updated in place and
 * read by the FLR kernels through flr_params.eps_device, so a training loop
 * needs no host read; state = device double[6], zero before the first
 * step: Adam moments of log eps (0, 1) and of log eps_mul (2, 3), and the
 * step count (4; its own count, independent of the network's optimizer);
 * dreg = the adjoint's per-crop gradients [n][2] (dL/deps, dL/deps_mul, as
 * flr_denoise_backward writes them), summed in crop order. With g the sum
 * times e (the derivative with respect to log e) and t the new step count:
 *   m <- beta1 m + (1 - beta1) g,   v <- beta2 v + (1 - beta2) g^2
 *   e <- e exp(-lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + adam_eps))
 * for eps, and for eps_mul when learn_mul is 1 and eps_mul > 0 (a zero
 * eps_mul stays zero). FP64 arithmetic, one thread. FLR_ERR_NULL,
 * FLR_ERR_ALIGN (reg 4-byte, state and dreg 8-byte aligned), FLR_ERR_SHAPE
 * for n < 1, FLR_ERR_MODE for learn_mul not 0 or 1, FLR_ERR_EPS for a
 * negative or non-finite hyperparameter or beta >= 1, FLR_ERR_ALIAS when two
 * of the arrays overlap. */
flr_status flr_reg_adam_step(float* reg, double* state, const double* dreg, int32_t n,
                             float lr, float beta1, float beta2, float adam_eps,
                             int32_t learn_mul, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* FLR_TRAIN_H */
