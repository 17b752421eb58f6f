// The two element-wise stages of an FLNR training step around the network
// and regression gradients: the L1 loss and its gradient (the training loss
// of the workload; Sec. 3.3 trains FLNR end to end on an image loss), and the
// AdamW update of the FP32 master weights (Adam with weight decay decoupled
// from the gradient, as published by Loshchilov and Hutter).
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <mutex>

#include "flr.h"
#include "flr_train.h"

namespace flrtrain {

constexpr int kBlock = 256;
constexpr int kMaxBlocks = 1024;

struct L1Args {
  const float* out;
  const float* target;
  float* grad;
  double* part;  // [nblocks]
  int64_t n;
  float scale;
};

// grad = scale sign(out - target); each workgroup's FP64 sum of
// |out - target| over a grid-stride range, added in thread order.
__global__ void __launch_bounds__(kBlock) l1_kernel(L1Args a) {
  __shared__ double red[kBlock];
  double s = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n; i += stride) {
    const float d = a.out[i] - a.target[i];
    a.grad[i] = d > 0.f ? a.scale : (d < 0.f ? -a.scale : 0.f);
    s += fabs((double)a.out[i] - (double)a.target[i]);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h /= 2) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.part[blockIdx.x] = red[0];
}

struct L1SumArgs {
  const double* part;
  int nblocks;
  double scale;
  double* loss;
};

// One workgroup: strided partial sums per thread, then a tree, both in a
// fixed order.
__global__ void __launch_bounds__(kBlock) l1_sum_kernel(L1SumArgs a) {
  __shared__ double red[kBlock];
  double s = 0.0;
  for (int b = threadIdx.x; b < a.nblocks; b += kBlock) s += a.part[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h /= 2) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.loss[0] = a.scale * red[0];
}

struct AdamWArgs {
  float* p;
  const float* g;
  float* m;
  float* v;
  int64_t n;
  float lr, beta1, beta2, eps, decay;  // decay = lr * weight_decay
  float step_size;                     // lr / (1 - beta1^t)
  float inv_sqrt_bc2;                  // 1 / sqrt(1 - beta2^t)
};

__global__ void __launch_bounds__(kBlock) adamw_kernel(AdamWArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= a.n) return;
  const float g = a.g[i];
  float p = a.p[i];
  p -= a.decay * p;
  const float m = a.beta1 * a.m[i] + (1.f - a.beta1) * g;
  const float v = a.beta2 * a.v[i] + (1.f - a.beta2) * g * g;
  a.m[i] = m;
  a.v[i] = v;
  const float denom = sqrtf(v) * a.inv_sqrt_bc2 + a.eps;
  a.p[i] = p - a.step_size * (m / denom);
}

// Adam on the logarithms of FLR's regularisers (eps, eps_mul), one thread:
// the adjoint's per-crop FP64 gradients summed in crop order, the chain
// factor of the logarithm (dL/dlog e = e dL/de), then Adam with its own
// step count t (state[4]) and moments (state[0..1] for eps, [2..3] for
// eps_mul); e <- e exp(-lr mhat / (sqrt(vhat) + adam_eps)).
struct RegAdamArgs {
  float* reg;
  double* state;
  const double* dreg;
  int n;
  int learn_mul;
  double lr, beta1, beta2, adam_eps;
};
__global__ void __launch_bounds__(64) reg_adam_kernel(RegAdamArgs a) {
  if (threadIdx.x != 0) return;
  double ge = 0.0, gm = 0.0;
  for (int k = 0; k < a.n; ++k) {
    ge += a.dreg[2 * k];
    gm += a.dreg[2 * k + 1];
  }
  const double t = a.state[4] + 1.0;
  a.state[4] = t;
  const double bc1 = 1.0 - pow(a.beta1, t), bc2 = 1.0 - pow(a.beta2, t);
  for (int j = 0; j < 2; ++j) {
    const double e = (double)a.reg[j];
    if (j == 1 && !(a.learn_mul && e > 0.0)) break;
    const double g = (j == 0 ? ge : gm) * e;
    const double m = a.beta1 * a.state[2 * j] + (1.0 - a.beta1) * g;
    const double v = a.beta2 * a.state[2 * j + 1] + (1.0 - a.beta2) * g * g;
    a.state[2 * j] = m;
    a.state[2 * j + 1] = v;
    a.reg[j] = (float)(e * exp(-a.lr * (m / bc1) / (sqrt(v / bc2) + a.adam_eps)));
  }
}

inline int l1_blocks(int64_t n) {
  const int64_t b = (n + kBlock - 1) / kBlock;
  return (int)(b < kMaxBlocks ? (b < 1 ? 1 : b) : kMaxBlocks);
}
inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
inline bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
  return a0 < b0 + nb && b0 < a0 + na;
}
constexpr int64_t kMaxElems = (int64_t)1 << 34;

// flr_l1_loss_grad_noalloc's partial sums: at most kMaxBlocks doubles
// (8 KiB), one copy per GPU, held until the process ends. Host code never
// passes the array's name to a kernel (on the host it is only a stand-in);
// it resolves the array's device address once per device and uses that.
static __device__ __align__(256) double scratch[kMaxBlocks];
constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices];

// Device address of `scratch` on the current device (resolved on the first
// call made with that device current).
hipError_t scratch_address(double** addr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_addr[dev] = p;
  }
  *addr = static_cast<double*>(g_scratch_addr[dev]);
  return hipSuccess;
}

// Argument checks shared by both L1 entry points: sizes, pointers and the
// scale (l1_check), then overlaps of the outputs with the inputs (l1_alias).
flr_status l1_check(int64_t n, const float* out, const float* target, float scale, float* grad,
                    double* loss) {
  if (n < 1 || n > kMaxElems) return FLR_ERR_SHAPE;
  if (!out || !target || !grad || !loss) return FLR_ERR_NULL;
  if (!aligned16(out) || !aligned16(target) || !aligned16(grad) ||
      (reinterpret_cast<uintptr_t>(loss) & 7u) != 0)
    return FLR_ERR_ALIGN;
  if (!(scale == scale) || scale == __builtin_huge_valf() || scale == -__builtin_huge_valf())
    return FLR_ERR_EPS;
  return FLR_OK;
}
flr_status l1_alias(int64_t n, const float* out, const float* target, float* grad, double* loss) {
  const size_t fb = (size_t)n * sizeof(float);
  if (overlaps(grad, fb, out, fb) || overlaps(grad, fb, target, fb) ||
      overlaps(loss, sizeof(double), out, fb) || overlaps(loss, sizeof(double), target, fb) ||
      overlaps(loss, sizeof(double), grad, fb))
    return FLR_ERR_ALIAS;
  return FLR_OK;
}

// The two launches, partial sums in `part` (l1_blocks(n) doubles).
flr_status l1_launch(int64_t n, const float* out, const float* target, float scale, float* grad,
                     double* loss, double* part, hipStream_t s) {
  const int nb = l1_blocks(n);
  const L1Args a = {out, target, grad, part, n, scale};
  hipLaunchKernelGGL(l1_kernel, dim3(nb), dim3(kBlock), 0, s, a);
  if (hipGetLastError() != hipSuccess) return FLR_ERR_HIP;
  const L1SumArgs b = {part, nb, (double)scale, loss};
  hipLaunchKernelGGL(l1_sum_kernel, dim3(1), dim3(kBlock), 0, s, b);
  return hipGetLastError() == hipSuccess ? FLR_OK : FLR_ERR_HIP;
}

}  // namespace flrtrain

using namespace flrtrain;

extern "C" {

size_t flr_l1_workspace_bytes(int64_t n) {
  if (n < 1 || n > kMaxElems) return 0;
  return (size_t)l1_blocks(n) * sizeof(double);
}

flr_status flr_l1_loss_grad(int64_t n, const float* out, const float* target, float scale,
                            float* grad, double* loss, void* workspace, size_t workspace_bytes,
                            void* stream) {
  flr_status st = l1_check(n, out, target, scale, grad, loss);
  if (st != FLR_OK) return st;
  const size_t need = flr_l1_workspace_bytes(n);
  if (!workspace || workspace_bytes < need) return FLR_ERR_WORKSPACE;
  if (!aligned16(workspace)) return FLR_ERR_ALIGN;
  if ((st = l1_alias(n, out, target, grad, loss)) != FLR_OK) return st;
  const size_t fb = (size_t)n * sizeof(float);
  if (overlaps(workspace, need, out, fb) || overlaps(workspace, need, target, fb) ||
      overlaps(workspace, need, grad, fb) || overlaps(workspace, need, loss, sizeof(double)))
    return FLR_ERR_ALIAS;
  return l1_launch(n, out, target, scale, grad, loss, static_cast<double*>(workspace),
                   reinterpret_cast<hipStream_t>(stream));
}

flr_status flr_l1_loss_grad_noalloc(int64_t n, const float* out, const float* target,
                                    float scale, float* grad, double* loss, void* stream) {
  flr_status st = l1_check(n, out, target, scale, grad, loss);
  if (st != FLR_OK) return st;
  if ((st = l1_alias(n, out, target, grad, loss)) != FLR_OK) return st;
  if (l1_blocks(n) > kMaxBlocks) return FLR_ERR_SHAPE;  // never for n <= 2^34
  double* part = nullptr;
  if (scratch_address(&part) != hipSuccess) return FLR_ERR_HIP;
  return l1_launch(n, out, target, scale, grad, loss, part, reinterpret_cast<hipStream_t>(stream));
}

flr_status flr_reg_adam_step(float* reg, double* state, const double* dreg, int32_t n,
                             float lr, float beta1, float beta2, float adam_eps,
                             int32_t learn_mul, void* stream) {
  if (!reg || !state || !dreg) return FLR_ERR_NULL;
  if ((reinterpret_cast<uintptr_t>(reg) & 3u) || (reinterpret_cast<uintptr_t>(state) & 7u) ||
      (reinterpret_cast<uintptr_t>(dreg) & 7u))
    return FLR_ERR_ALIGN;
  if (n < 1) return FLR_ERR_SHAPE;
  if (learn_mul != 0 && learn_mul != 1) return FLR_ERR_MODE;
  const float hp[4] = {lr, beta1, beta2, adam_eps};
  for (float x : hp)
    if (!(x >= 0.f) || x == __builtin_huge_valf()) return FLR_ERR_EPS;
  if (!(beta1 < 1.f) || !(beta2 < 1.f)) return FLR_ERR_EPS;
  if (overlaps(reg, 2 * sizeof(float), state, 6 * sizeof(double)) ||
      overlaps(reg, 2 * sizeof(float), dreg, 2 * (size_t)n * sizeof(double)) ||
      overlaps(state, 6 * sizeof(double), dreg, 2 * (size_t)n * sizeof(double)))
    return FLR_ERR_ALIAS;
  const RegAdamArgs a = {reg, state, dreg, n, learn_mul, lr, beta1, beta2, adam_eps};
  hipLaunchKernelGGL(reg_adam_kernel, dim3(1), dim3(64), 0, reinterpret_cast<hipStream_t>(stream),
                     a);
  return hipGetLastError() == hipSuccess ? FLR_OK : FLR_ERR_HIP;
}

flr_status flr_adamw_step(int64_t n, float* params, const float* grads, float* m, float* v,
                          int32_t step, float lr, float beta1, float beta2, float eps,
                          float weight_decay, void* stream) {
  if (n < 1 || n > kMaxElems) return FLR_ERR_SHAPE;
  if (!params || !grads || !m || !v) return FLR_ERR_NULL;
  if (!aligned16(params) || !aligned16(grads) || !aligned16(m) || !aligned16(v))
    return FLR_ERR_ALIGN;
  if (step < 1) return FLR_ERR_MODE;
  const float hp[5] = {lr, beta1, beta2, eps, weight_decay};
  for (float x : hp)
    if (!(x >= 0.f) || x == __builtin_huge_valf()) return FLR_ERR_EPS;
  if (!(beta1 < 1.f) || !(beta2 < 1.f)) return FLR_ERR_EPS;
  const size_t fb = (size_t)n * sizeof(float);
  const void* bufs[4] = {params, grads, m, v};
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j)
      if (overlaps(bufs[i], fb, bufs[j], fb)) return FLR_ERR_ALIAS;
  const double bc1 = 1.0 - __builtin_pow((double)beta1, (double)step);
  const double bc2 = 1.0 - __builtin_pow((double)beta2, (double)step);
  AdamWArgs a = {};
  a.p = params;
  a.g = grads;
  a.m = m;
  a.v = v;
  a.n = n;
  a.lr = lr;
  a.beta1 = beta1;
  a.beta2 = beta2;
  a.eps = eps;
  a.decay = (float)((double)lr * weight_decay);
  a.step_size = (float)(lr / bc1);
  a.inv_sqrt_bc2 = (float)(1.0 / __builtin_sqrt(bc2));
  hipLaunchKernelGGL(adamw_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     reinterpret_cast<hipStream_t>(stream), a);
  return hipGetLastError() == hipSuccess ? FLR_OK : FLR_ERR_HIP;
}

}  // extern "C"
