"""ctypes view of ``libflr.so`` (the C ABI in ``include/flr.h``).

Only argument marshalling happens here; every step of the path runs in the
library's HIP kernels. The library must have been built in-tree (see
``paper_2410_11625_amd/build.py``); if it is missing, loading fails loudly
and nothing falls back to any other implementation.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libflr.so")

FLR_OK = 0
FLR_REG_RIDGE = 0
FLR_REG_PAPER = 1
FLR_FLAG_RAW_MOMENTS = 1
FLR_FLAG_INTERCEPT_PAIR = 2
FLR_MAX_GUIDES = 12
FLR_MAX_CHANNELS = 4
FLR_MAX_RADIUS = 32

STATUS_NAMES = {
    0: "FLR_OK", 1: "FLR_ERR_NULL", 2: "FLR_ERR_SHAPE", 3: "FLR_ERR_RADIUS", 4: "FLR_ERR_EPS",
    5: "FLR_ERR_CHANNELS", 6: "FLR_ERR_ALIAS", 7: "FLR_ERR_ALIGN", 8: "FLR_ERR_WORKSPACE",
    9: "FLR_ERR_MODE", 10: "FLR_ERR_HIP",
}

# Every symbol include/flr.h declares.
EXPORTED = ("flr_num_moment_planes", "flr_num_coeff_planes", "flr_denoise_workspace_bytes",
            "flr_moments", "flr_solve", "flr_coefficients", "flr_apply", "flr_denoise",
            "flr_status_str", "flr_validate_params", "flr_denoise_backward_workspace_bytes",
            "flr_denoise_backward", "flr_lowres_workspace_bytes", "flr_denoise_lowres",
            "flr_batch_workspace_bytes", "flr_batch_plan", "flr_batch_run", "flr_batch_failed",
            # include/flr_net.h
            "flr_net_num_params", "flr_net_packed_bytes", "flr_net_pack", "flr_net_workspace_bytes",
            "flr_net_forward", "flr_net_backward_workspace_bytes", "flr_net_backward",
            "flr_flnr_workspace_bytes", "flr_flnr_denoise", "flr_net_trace_bytes",
            "flr_net_trace_tensor", "flr_net_forward_trace",
            # include/flr_train.h
            "flr_l1_workspace_bytes", "flr_l1_loss_grad", "flr_adamw_step",
            "flr_l1_loss_grad_noalloc", "flr_reg_adam_step")


class FlrParams(ctypes.Structure):
    _fields_ = [
        ("height", ctypes.c_int32),
        ("width", ctypes.c_int32),
        ("num_guides", ctypes.c_int32),
        ("num_channels", ctypes.c_int32),
        ("radius", ctypes.c_int32),
        ("eps", ctypes.c_float),
        ("eps_mul", ctypes.c_float),
        ("reg_mode", ctypes.c_int32),
        ("average_coeffs", ctypes.c_int32),
        ("fused", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("tile_rows", ctypes.c_int32),
        ("eps_device", ctypes.c_void_p),
    ]


FLR_BATCH_MAX = 64


class FlrFrame(ctypes.Structure):
    """flr_frame: one frame of a batch."""
    _fields_ = [
        ("height", ctypes.c_int32),
        ("width", ctypes.c_int32),
        ("noisy_height", ctypes.c_int32),
        ("noisy_width", ctypes.c_int32),
        ("tile_rows", ctypes.c_int32),
        ("apply_rows", ctypes.c_int32),
        ("guides", ctypes.c_void_p),
        ("guides_low", ctypes.c_void_p),
        ("noisy", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
    ]


class FlrBatch(ctypes.Structure):
    """flr_batch: a planned batch (filled by flr_batch_plan)."""
    _fields_ = [
        ("params", FlrParams),
        ("num_frames", ctypes.c_int32),
        ("num_joint", ctypes.c_int32),
        ("coeff_blocks", ctypes.c_int32),
        ("apply_blocks", ctypes.c_int32),
        ("up_blocks", ctypes.c_int32),
        ("persistent_blocks", ctypes.c_int32),
        ("num_items", ctypes.c_int32),
        ("walk_table", ctypes.c_void_p),
        ("apply_table", ctypes.c_void_p),
        ("up_table", ctypes.c_void_p),
        ("walk_starts", ctypes.c_void_p),
        ("persistent_plan", ctypes.c_void_p),
        ("joint_guides", ctypes.c_void_p * FLR_BATCH_MAX),
        ("joint_noisy", ctypes.c_void_p * FLR_BATCH_MAX),
        ("joint_sums", ctypes.c_void_p * FLR_BATCH_MAX),
        ("joint_models", ctypes.c_void_p * FLR_BATCH_MAX),
        ("joint_mean", ctypes.c_void_p * FLR_BATCH_MAX),
        ("joint_height", ctypes.c_int32 * FLR_BATCH_MAX),
        ("joint_width", ctypes.c_int32 * FLR_BATCH_MAX),
    ]


class FLRError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = int(status)
        name = STATUS_NAMES.get(self.status, str(status))
        msg = f"{name}: {status_str(self.status)}"
        super().__init__(f"{what}: {msg}" if what else msg)


_lib = None


def lib() -> ctypes.CDLL:
    """Load the library once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libflr.so not found at {LIB_PATH}; build it with "
                          "`python -m paper_2410_11625_amd.build` (there is no fallback)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(FlrParams)
    vp = ctypes.c_void_p
    L.flr_num_moment_planes.argtypes = [ctypes.c_int32, ctypes.c_int32]
    L.flr_num_moment_planes.restype = ctypes.c_size_t
    L.flr_num_coeff_planes.argtypes = [ctypes.c_int32, ctypes.c_int32]
    L.flr_num_coeff_planes.restype = ctypes.c_size_t
    L.flr_denoise_workspace_bytes.argtypes = [P]
    L.flr_denoise_workspace_bytes.restype = ctypes.c_size_t
    L.flr_validate_params.argtypes = [P]
    L.flr_validate_params.restype = ctypes.c_int
    L.flr_moments.argtypes = [P, vp, vp, vp, vp]
    L.flr_moments.restype = ctypes.c_int
    L.flr_solve.argtypes = [P, vp, vp, vp]
    L.flr_solve.restype = ctypes.c_int
    L.flr_coefficients.argtypes = [P, vp, vp, vp, vp]
    L.flr_coefficients.restype = ctypes.c_int
    L.flr_apply.argtypes = [P, vp, vp, vp, vp]
    L.flr_apply.restype = ctypes.c_int
    L.flr_denoise.argtypes = [P, vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.flr_denoise.restype = ctypes.c_int
    L.flr_denoise_backward_workspace_bytes.argtypes = [P]
    L.flr_denoise_backward_workspace_bytes.restype = ctypes.c_size_t
    L.flr_denoise_backward.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.flr_denoise_backward.restype = ctypes.c_int
    L.flr_lowres_workspace_bytes.argtypes = [P, ctypes.c_int32, ctypes.c_float, ctypes.c_int32]
    L.flr_lowres_workspace_bytes.restype = ctypes.c_size_t
    L.flr_denoise_lowres.argtypes = [P, ctypes.c_int32, ctypes.c_float, ctypes.c_int32, vp, vp, vp,
                                     vp, ctypes.c_size_t, vp]
    L.flr_denoise_lowres.restype = ctypes.c_int
    F = ctypes.POINTER(FlrFrame)
    Bp = ctypes.POINTER(FlrBatch)
    L.flr_batch_workspace_bytes.argtypes = [P, F, ctypes.c_int32]
    L.flr_batch_workspace_bytes.restype = ctypes.c_size_t
    L.flr_batch_plan.argtypes = [P, F, ctypes.c_int32, vp, ctypes.c_size_t, Bp]
    L.flr_batch_plan.restype = ctypes.c_int
    L.flr_batch_run.argtypes = [Bp, vp]
    L.flr_batch_run.restype = ctypes.c_int
    L.flr_batch_failed.argtypes = [Bp, ctypes.POINTER(ctypes.c_int32)]
    L.flr_batch_failed.restype = ctypes.c_int
    L.flr_net_num_params.restype = ctypes.c_size_t
    L.flr_net_packed_bytes.restype = ctypes.c_size_t
    L.flr_net_pack.argtypes = [vp, vp, vp]
    L.flr_net_pack.restype = ctypes.c_int
    L.flr_net_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
    L.flr_net_workspace_bytes.restype = ctypes.c_size_t
    L.flr_net_forward.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, vp,
                                  ctypes.c_size_t, vp]
    L.flr_net_forward.restype = ctypes.c_int
    L.flr_net_trace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
    L.flr_net_trace_bytes.restype = ctypes.c_size_t
    i32p = ctypes.POINTER(ctypes.c_int32)
    L.flr_net_trace_tensor.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_size_t), i32p, i32p, i32p]
    L.flr_net_trace_tensor.restype = ctypes.c_int
    L.flr_net_forward_trace.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, vp,
                                        ctypes.c_size_t, vp]
    L.flr_net_forward_trace.restype = ctypes.c_int
    L.flr_net_backward_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
    L.flr_net_backward_workspace_bytes.restype = ctypes.c_size_t
    L.flr_net_backward.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, vp, vp,
                                   ctypes.c_int32, vp, ctypes.c_size_t, vp]
    L.flr_net_backward.restype = ctypes.c_int
    L.flr_flnr_workspace_bytes.argtypes = [P]
    L.flr_flnr_workspace_bytes.restype = ctypes.c_size_t
    L.flr_flnr_denoise.argtypes = [P, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.flr_flnr_denoise.restype = ctypes.c_int
    L.flr_l1_workspace_bytes.argtypes = [ctypes.c_int64]
    L.flr_l1_workspace_bytes.restype = ctypes.c_size_t
    L.flr_l1_loss_grad.argtypes = [ctypes.c_int64, vp, vp, ctypes.c_float, vp, vp, vp,
                                   ctypes.c_size_t, vp]
    L.flr_l1_loss_grad.restype = ctypes.c_int
    L.flr_l1_loss_grad_noalloc.argtypes = [ctypes.c_int64, vp, vp, ctypes.c_float, vp, vp, vp]
    L.flr_l1_loss_grad_noalloc.restype = ctypes.c_int
    L.flr_reg_adam_step.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, ctypes.c_float, ctypes.c_int32, vp]
    L.flr_reg_adam_step.restype = ctypes.c_int
    f = ctypes.c_float
    L.flr_adamw_step.argtypes = [ctypes.c_int64, vp, vp, vp, vp, ctypes.c_int32, f, f, f, f, f, vp]
    L.flr_adamw_step.restype = ctypes.c_int
    L.flr_status_str.argtypes = [ctypes.c_int]
    L.flr_status_str.restype = ctypes.c_char_p
    _lib = L
    return L


def status_str(status: int) -> str:
    try:
        return lib().flr_status_str(int(status)).decode()
    except ImportError:
        return STATUS_NAMES.get(int(status), "unknown")


def check(status: int, what: str = "") -> None:
    if status != FLR_OK:
        raise FLRError(status, what)
