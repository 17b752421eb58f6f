/*
 * flr_net.h - C ABI of the FLNR guide network and of FLNR denoising.
 *
 * Fast Local Neural Regression (Sec. 3.3) runs a small U-Net over the
 * guides and the noisy input and feeds its output channels to the
 * regression as additional guides. This library implements the
 * configuration's three-level variant, with BF16 weights and activations
 * and FP32 accumulation on the matrix cores:
 *
 *   input   8 guides then 3 noisy channels (11 channels, planar FP32), each
 *           value v compressed to sign(v) log(1 + |v|)
 *   in3     3x3 conv 11 -> 16, ReLU        } full resolution
 *   in1     1x1 conv 16 -> 16, ReLU  = e0  }
 *   e1a     3x3 conv 16 -> 32, ReLU
 *   e1b     3x3 conv 32 -> 32, stride 2, ReLU = e1      (half resolution)
 *   e2a     3x3 conv 32 -> 64, ReLU
 *   e2b     3x3 conv 64 -> 64, stride 2, ReLU = e2      (quarter resolution)
 *   d1a     3x3 conv [up2(e2), e1] 96 -> 32, ReLU
 *   d1b     3x3 conv 32 -> 32, ReLU = d1
 *   d0a     3x3 conv [up2(d1), e0] 48 -> 16, ReLU
 *   d0b     3x3 conv 16 -> 16, ReLU
 *   out3    3x3 conv 16 -> 16, ReLU
 *   out1    1x1 conv 16 -> 4, sigmoid      -> 4 extra guide planes (FP32)
 *
 * Convolutions are cross-correlations with zero padding k/2 and a bias; a
 * stride-2 layer samples input (2i, 2j) and gives ceil(n/2) outputs; up2 is
 * nearest upsampling cropped to the skip's size; [a, b] concatenates
 * channels in that order. Weights, biases, the input and every activation
 * between layers are rounded to BF16 (nearest, ties to even); products are
 * accumulated in FP32; the sigmoid output is FP32.
 *
 * Parameters: one FP32 vector, layer by layer in the order above, each layer
 * its weight [c_out][c_in][k][k] (row-major) then its bias [c_out];
 * flr_net_num_params() elements in all. flr_net_pack() turns it into the
 * device-side BF16 form the kernels read (once per set of weights).
 *
 * Ownership and errors as in flr.h: every pointer is caller-owned device
 * memory, 16-byte aligned; the library never allocates; arguments are
 * checked on the host before any launch; FLR_ERR_HIP on launch failure.
 */
#ifndef FLR_NET_H
#define FLR_NET_H

#include <stddef.h>
#include <stdint.h>

#include "flr.h"

#ifdef __cplusplus
extern "C" {
#endif

#define FLR_NET_IN_GUIDES 8   /* guide planes the network reads */
#define FLR_NET_IN_NOISY 3    /* noisy planes the network reads */
#define FLR_NET_OUT 4         /* extra guide planes it writes */

/* Number of FP32 parameters (weights and biases of all layers). */
size_t flr_net_num_params(void);

/* Bytes of the packed (device) parameter block. */
size_t flr_net_packed_bytes(void);

/* params: device FP32 [flr_net_num_params()]; packed: device buffer of
 * flr_net_packed_bytes(). Rounds to BF16 and reorders into the matrix-core
 * operand layout. */
flr_status flr_net_pack(const float* params, void* packed, void* stream);

/* Workspace bytes of flr_net_forward for a height x width frame (the
 * intermediate activations, BF16). 0 for invalid sizes. */
size_t flr_net_workspace_bytes(int32_t height, int32_t width);

/* guides [8][H][W], noisy [3][H][W] (planar FP32) -> out [4][H][W] (FP32,
 * in (0, 1)). packed from flr_net_pack. FLR_ERR_SHAPE for sizes outside
 * 1..FLR_MAX_DIM or more than 2^28 pixels, FLR_ERR_WORKSPACE when the
 * workspace is missing or smaller than flr_net_workspace_bytes, FLR_ERR_ALIAS
 * when out or the workspace overlaps an input. */
flr_status flr_net_forward(int32_t height, int32_t width, const float* guides,
                           const float* noisy, const void* packed, float* out,
                           void* workspace, size_t workspace_bytes, void* stream);

/* Verification view of one forward pass (Sec. 3.3's network, layer by
 * layer): flr_net_forward_trace computes exactly what flr_net_forward
 * computes, with the same kernels, and leaves every layer's BF16 output
 * activation in the caller-owned trace buffer, so that each layer can be
 * checked on the inputs the device actually fed it. Trace tensor index:
 *   0 x0 (the prepared input: 11 compressed channels, 5 zero)   1 in3
 *   2 in1 (= e0)   3 e1a   4 e1b (= e1)   5 e2a   6 e2b (= e2)   7 d1a
 *   8 d1b (= d1)   9 d0a   10 d0b   11 out3
 * (out1's sigmoid output is `out`, as in flr_net_forward). Each tensor is
 * HWC BF16 (uint16 bit patterns): [h][w][channels], channels a multiple of
 * 16 (x0 pads 11 to 16 with zeros). */
size_t flr_net_trace_bytes(int32_t height, int32_t width);

/* Where trace tensor `index` (0..11) lives in the trace buffer of a height x
 * width frame: byte offset, channel count and grid (full, half or quarter
 * resolution: ceil(n/2) per halving). FLR_ERR_SHAPE for invalid sizes,
 * FLR_ERR_NULL for a null output pointer, FLR_ERR_MODE for an index out of
 * range. Host only. */
flr_status flr_net_trace_tensor(int32_t height, int32_t width, int32_t index, size_t* offset,
                                int32_t* channels, int32_t* tensor_height, int32_t* tensor_width);

/* flr_net_forward with the trace buffer (flr_net_trace_bytes, 16-byte
 * aligned, caller-owned device memory) in place of the workspace. Errors as
 * flr_net_forward (FLR_ERR_WORKSPACE when the trace buffer is missing or too
 * small). */
flr_status flr_net_forward_trace(int32_t height, int32_t width, const float* guides,
                                 const float* noisy, const void* packed, float* out, void* trace,
                                 size_t trace_bytes, void* stream);

/* Workspace bytes of flr_net_backward for a height x width frame: the
 * forward's activations plus FP32 gradient tensors (about 1.3 KB per pixel).
 * 0 for invalid sizes. */
size_t flr_net_backward_workspace_bytes(int32_t height, int32_t width);

/* Gradient of a loss with respect to every network parameter, given the
 * loss's gradient grad_out [4][H][W] (planar FP32) with respect to the four
 * sigmoid outputs of flr_net_forward on the same guides and noisy input
 * (Sec. 3.3: the network is trained by backpropagating the denoising loss
 * through the regression into it; the regression's part is
 * flr_denoise_backward, whose guide gradient planes 8..11 are grad_out).
 *
 * The call reruns the forward (it keeps no state between calls), then
 * reverses the layers. BF16 rounding in the forward is treated as the
 * identity (straight-through): the result is the gradient of the exact
 * network at the BF16 weights and activations, accumulated in FP32.
 *
 * params: the FP32 parameters packed has been made from (flr_net_pack), in
 * the layout of flr_net_num_params(). grad_params [flr_net_num_params()]
 * receives the gradients in the same layout, overwritten when accumulate is
 * 0 and added to when 1 (to sum a batch frame by frame); the weight
 * gradients are sums over all pixels, added in a fixed order (repeatable
 * bit for bit). Errors as flr_net_forward, FLR_ERR_MODE for accumulate not
 * 0 or 1, FLR_ERR_ALIAS when grad_params or the workspace overlaps an input
 * or each other. Tuning: the data gradients take 16 input channels per
 * thread on layers of at least FLR_DGRAD_WIDE_PX pixels (environment
 * variable, read at each call; default 2^18) and 8 below; the result is
 * bit-identical either way. */
flr_status flr_net_backward(int32_t height, int32_t width, const float* guides,
                            const float* noisy, const float* params, const void* packed,
                            const float* grad_out, float* grad_params, int32_t accumulate,
                            void* workspace, size_t workspace_bytes, void* stream);

/* Workspace bytes of flr_flnr_denoise for params p (p->num_guides must be
 * FLR_NET_IN_GUIDES + FLR_NET_OUT = 12 and p->num_channels 3). */
size_t flr_flnr_workspace_bytes(const flr_params* p);

/* FLNR: the network, then FLR over the 12 guides (Sec. 3.3 with the
 * configuration's appended-guide form). guides12 is [12][H][W]: the caller
 * fills planes 0..7 with the input guides; the network's 4 planes are
 * written to planes 8..11, then flr_denoise(p) runs on all 12. noisy [3][H][W],
 * out [3][H][W]. p selects the regression path and its parameters as in
 * flr_denoise. */
flr_status flr_flnr_denoise(const flr_params* p, float* guides12, const float* noisy,
                            const void* packed, float* out, void* workspace,
                            size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* FLR_NET_H */
