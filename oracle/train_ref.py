"""FP64 reference of the element-wise training-step stages -- TEST
INFRASTRUCTURE ONLY.

Only the tests, the package's smoke check and the benchmark's CPU-baseline
leg may use this module; the product path never imports it.

* L1 loss of the denoised output against the target, the workload's training
  loss (Sec. 3.3 trains FLNR end to end on an image loss): loss = scale *
  sum |out - target|, gradient scale * sign(out - target), sign(0) = 0.
* AdamW (Adam with weight decay decoupled from the gradient, Loshchilov and
  Hutter): the update of the FP32 master weights, written from its published
  definition with bias-corrected first and second moments.
* Adam on the logarithm of a positive regulariser (the Appendix learns its
  regularisers by backpropagation): the parameter is log e, its gradient e
  times dL/de, and e the exponential of the updated logarithm.
"""
from __future__ import annotations

import numpy as np

__all__ = ["l1_loss_grad", "adamw_step", "log_adam_step"]


def l1_loss_grad(out, target, scale: float):
    """(loss, grad): loss in FP64; the sign is taken of the FP32 difference
    when both inputs are FP32 (as a kernel working on FP32 data does)."""
    out = np.asarray(out)
    target = np.asarray(target)
    d = out - target
    loss = float(scale) * float(np.sum(np.abs(out.astype(np.float64) - target.astype(np.float64))))
    return loss, float(scale) * np.sign(d).astype(np.float64)


def adamw_step(p, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
               eps: float = 1e-8, weight_decay: float = 0.0):
    """One AdamW update; returns new (p, m, v) as float64 arrays. step t >= 1."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    p = p * (1.0 - lr * weight_decay)
    p = p - lr * m_hat / (np.sqrt(v_hat) + eps)
    return p, m, v


def log_adam_step(e: float, grad_e: float, m: float, v: float, step: int, lr: float,
                  beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-12):
    """One Adam update of log(e) for a loss gradient grad_e = dL/de; returns
    (new e, m, v). The update of log e is an AdamW update without decay of
    the parameter log e with gradient e * grad_e."""
    logp, m2, v2 = adamw_step(np.log(e), e * grad_e, m, v, step, lr, beta1, beta2, eps, 0.0)
    return float(np.exp(logp)), float(m2), float(v2)
