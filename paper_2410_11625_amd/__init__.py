"""Fast Local Regression (FLR) on AMD MI355X (gfx950).

The windowed per-pixel regularised linear regression of "Fast Local Neural
Regression for Low-Cost, Path Traced Lambertian Global Illumination"
(Sec. 3.1-3.2 and the Appendix) and the FLNR guide network (Sec. 3.3), as
hand-written HIP kernels behind the C ABI in ``include/flr.h`` and
``include/flr_net.h``. This package is the thin Python binding.
"""
from .api import (PATHS, Batch, FLNRTrainer, FLRError, adamw_step, apply, backward_workspace_bytes, coefficients, denoise,
                  denoise_backward, denoise_lowres, flnr_denoise, flnr_workspace_bytes, flr,
                  l1_loss_grad, lowres_workspace_bytes, make_params, moments, net_backward, net_forward,
                  net_forward_trace, net_num_params, net_pack, reg_adam_step, num_coeff_planes, num_moment_planes, solve, workspace_bytes)

__all__ = ["PATHS", "Batch", "FLNRTrainer", "FLRError", "adamw_step", "l1_loss_grad", "apply", "backward_workspace_bytes", "coefficients", "denoise",
           "denoise_backward", "denoise_lowres", "flnr_denoise", "flnr_workspace_bytes", "flr",
           "lowres_workspace_bytes", "make_params",
           "moments", "net_backward", "net_forward", "net_forward_trace", "net_num_params", "net_pack", "reg_adam_step", "num_coeff_planes",
           "num_moment_planes", "solve", "workspace_bytes"]
