"""Python mirror of the C ABI on torch tensors.

Tensors are float32, contiguous, on a HIP device; they only provide memory
and the current stream. Every computation runs in ``libflr.so``.
Shapes: ``guides`` [Q,H,W] (without the implied constant guide), ``noisy``
[C,H,W], moments [M,H,W], coefficients [(Q+1)*C,H,W], output [C,H,W].
"""
from __future__ import annotations

import ctypes
import math

import torch

from ._lib import (FLR_BATCH_MAX, FLR_FLAG_INTERCEPT_PAIR, FLR_FLAG_RAW_MOMENTS, FLR_REG_PAPER, FLR_REG_RIDGE, FLRError,
                   FlrBatch, FlrFrame, FlrParams, check, lib)

_MODES = {"ridge": FLR_REG_RIDGE, "paper": FLR_REG_PAPER}
# flr_denoise execution paths (flr_path in the C header)
PATHS = {"stages": 0, "fused": 1, "two_pass": 2}


def _path(fused) -> int:
    """True/False keep their meaning (fused kernel / three stages); a path name
    or its integer value selects any path."""
    if isinstance(fused, str):
        return PATHS[fused]
    if isinstance(fused, bool):
        return 1 if fused else 0
    return int(fused)


def _need(t: torch.Tensor, name: str, ndim: int = 3) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32, got {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a HIP device (no CPU path exists)")
    if t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dims, got shape {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _stream(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _eps_device_ptr(eps_device):
    """Device address of a float32 tensor of 2 (eps, eps_mul), or None."""
    if eps_device is None:
        return None
    if not isinstance(eps_device, torch.Tensor) or eps_device.dtype != torch.float32 or \
            eps_device.device.type != "cuda" or eps_device.numel() < 2 or \
            not eps_device.is_contiguous():
        raise ValueError("eps_device must be a contiguous float32 device tensor of 2 elements")
    return eps_device.data_ptr()


def make_params(H: int, W: int, Q: int, C: int, radius: int, eps: float = 1e-3,
                mode: str = "ridge", eps_mul: float = 0.0, average: bool = True,
                fused=True, raw: bool = False, tile_rows: int = 0,
                eps_device: torch.Tensor | None = None,
                intercept_pair: bool = False) -> FlrParams:
    """flr_params; ``eps_device`` (float32 device tensor (eps, eps_mul)) makes
    the kernels read the regularisers from the device instead of eps and
    eps_mul."""
    if mode not in _MODES:
        raise ValueError(f"mode must be one of {sorted(_MODES)}")
    return FlrParams(height=H, width=W, num_guides=Q, num_channels=C, radius=radius,
                     eps=eps, eps_mul=eps_mul, reg_mode=_MODES[mode],
                     average_coeffs=int(bool(average)), fused=_path(fused),
                     flags=(FLR_FLAG_RAW_MOMENTS if raw else 0) |
                     (FLR_FLAG_INTERCEPT_PAIR if intercept_pair else 0), tile_rows=tile_rows,
                     eps_device=_eps_device_ptr(eps_device))


def num_moment_planes(Q: int, C: int) -> int:
    return int(lib().flr_num_moment_planes(Q, C))


def num_coeff_planes(Q: int, C: int) -> int:
    return int(lib().flr_num_coeff_planes(Q, C))


def workspace_bytes(p: FlrParams) -> int:
    return int(lib().flr_denoise_workspace_bytes(ctypes.byref(p)))


def moments(guides: torch.Tensor, noisy: torch.Tensor, radius: int, *, raw: bool = False,
            tile_rows: int = 0, out: torch.Tensor | None = None) -> torch.Tensor:
    """Window moments (central, or raw sums with ``raw``) as [M,H,W]."""
    _need(guides, "guides")
    _need(noisy, "noisy")
    Q, H, W = guides.shape
    C = noisy.shape[0]
    p = make_params(H, W, Q, C, radius, raw=raw, tile_rows=tile_rows)
    M = num_moment_planes(Q, C)
    if out is None:
        out = torch.empty((M, H, W), dtype=torch.float32, device=guides.device)
    _need(out, "out")
    check(lib().flr_moments(ctypes.byref(p), guides.data_ptr(), noisy.data_ptr(),
                            out.data_ptr(), _stream(guides)), "flr_moments")
    return out


def solve(moment_planes: torch.Tensor, num_guides: int, num_channels: int, eps: float = 1e-3,
          mode: str = "ridge", eps_mul: float = 0.0,
          out: torch.Tensor | None = None) -> torch.Tensor:
    """Per-pixel regularised solve: moment planes -> coefficient planes [(Q+1)*C,H,W]."""
    _need(moment_planes, "moments")
    _, H, W = moment_planes.shape
    Q, C = num_guides, num_channels
    if moment_planes.shape[0] != num_moment_planes(Q, C):
        raise ValueError("moment plane count does not match num_guides/num_channels")
    p = make_params(H, W, Q, C, 0, eps=eps, mode=mode, eps_mul=eps_mul)
    if out is None:
        out = torch.empty((num_coeff_planes(Q, C), H, W), dtype=torch.float32,
                          device=moment_planes.device)
    _need(out, "out")
    check(lib().flr_solve(ctypes.byref(p), moment_planes.data_ptr(), out.data_ptr(),
                          _stream(moment_planes)), "flr_solve")
    return out


def coefficients(guides: torch.Tensor, noisy: torch.Tensor, radius: int, eps: float = 1e-3,
                 mode: str = "ridge", eps_mul: float = 0.0, tile_rows: int = 0,
                 out: torch.Tensor | None = None, intercept_pair: bool = False) -> torch.Tensor:
    """Moments and solve in one pass -> coefficient planes [(Q+1)*C,H,W]
    (with ``intercept_pair``: [(Q+2)*C,H,W], the intercepts' lo parts last)."""
    _need(guides, "guides")
    _need(noisy, "noisy")
    Q, H, W = guides.shape
    C = noisy.shape[0]
    p = make_params(H, W, Q, C, radius, eps=eps, mode=mode, eps_mul=eps_mul, tile_rows=tile_rows,
                    intercept_pair=intercept_pair)
    if out is None:
        out = torch.empty((num_coeff_planes(Q, C) + (C if intercept_pair else 0), H, W),
                          dtype=torch.float32, device=guides.device)
    _need(out, "out")
    check(lib().flr_coefficients(ctypes.byref(p), guides.data_ptr(), noisy.data_ptr(),
                                 out.data_ptr(), _stream(guides)), "flr_coefficients")
    return out


def apply(guides: torch.Tensor, coeffs: torch.Tensor, radius: int, average: bool = True,
          tile_rows: int = 0, out: torch.Tensor | None = None,
          intercept_pair: bool = False) -> torch.Tensor:
    """Optional window-average of the coefficients, then reconstruction -> [C,H,W]."""
    _need(guides, "guides")
    _need(coeffs, "coeffs")
    Q, H, W = guides.shape
    F = Q + 2 if intercept_pair else Q + 1
    if coeffs.shape[0] % F != 0:
        raise ValueError(f"coefficient plane count must be a multiple of {F}")
    C = coeffs.shape[0] // F
    p = make_params(H, W, Q, C, radius, average=average, tile_rows=tile_rows,
                    intercept_pair=intercept_pair)
    if out is None:
        out = torch.empty((C, H, W), dtype=torch.float32, device=guides.device)
    _need(out, "out")
    check(lib().flr_apply(ctypes.byref(p), guides.data_ptr(), coeffs.data_ptr(),
                          out.data_ptr(), _stream(guides)), "flr_apply")
    return out


def denoise(noisy: torch.Tensor, guides: torch.Tensor, radius: int = 8, eps: float = 1e-3,
            mode: str = "ridge", eps_mul: float = 0.0, average: bool = True,
            fused=True, tile_rows: int = 0, out: torch.Tensor | None = None,
            workspace: torch.Tensor | None = None,
            eps_device: torch.Tensor | None = None) -> torch.Tensor:
    """The whole FLR path -> [C,H,W]. ``fused``: True (one kernel), False
    (three stages) or a path name from ``PATHS``. ``workspace`` is a uint8
    device tensor of at least ``workspace_bytes`` bytes; it is allocated when
    omitted. ``eps_device``: see make_params."""
    _need(guides, "guides")
    _need(noisy, "noisy")
    Q, H, W = guides.shape
    C = noisy.shape[0]
    if noisy.shape[1:] != guides.shape[1:]:
        raise ValueError("noisy and guides must have the same height and width")
    p = make_params(H, W, Q, C, radius, eps=eps, mode=mode, eps_mul=eps_mul, average=average,
                    fused=fused, tile_rows=tile_rows, eps_device=eps_device)
    need = workspace_bytes(p)
    if need == 0 and lib().flr_validate_params(ctypes.byref(p)) != 0:
        check(lib().flr_validate_params(ctypes.byref(p)), "flr_denoise")
    if workspace is None and need > 0:
        workspace = torch.empty(need, dtype=torch.uint8, device=guides.device)
    ws_ptr = workspace.data_ptr() if workspace is not None else None
    ws_len = workspace.numel() * workspace.element_size() if workspace is not None else 0
    if out is None:
        out = torch.empty((C, H, W), dtype=torch.float32, device=guides.device)
    _need(out, "out")
    check(lib().flr_denoise(ctypes.byref(p), guides.data_ptr(), noisy.data_ptr(), out.data_ptr(),
                            ws_ptr, ws_len, _stream(guides)), "flr_denoise")
    return out


# --------------------------------------------------------------------------
# The paper's fast variant (flr_denoise_lowres)


def lowres_workspace_bytes(p: FlrParams, block: int = 8, sigma_low: float = 1.25,
                           radius_low: int = 4) -> int:
    return int(lib().flr_lowres_workspace_bytes(ctypes.byref(p), block, sigma_low, radius_low))


def denoise_lowres(noisy: torch.Tensor, guides: torch.Tensor, block: int = 8,
                   sigma_low: float = 1.25, radius_low: int = 4, eps: float = 1e-3,
                   mode: str = "ridge", eps_mul: float = 0.0, out: torch.Tensor | None = None,
                   workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Block-downsampled moments, a low-resolution Gaussian blur (sigma_low,
    taps -radius_low..radius_low) and solve, bilinearly interpolated models
    -> [C,H,W]."""
    _need(guides, "guides")
    _need(noisy, "noisy")
    Q, H, W = guides.shape
    C = noisy.shape[0]
    if noisy.shape[1:] != guides.shape[1:]:
        raise ValueError("noisy and guides must have the same height and width")
    p = make_params(H, W, Q, C, 0, eps=eps, mode=mode, eps_mul=eps_mul, average=False)
    need = lowres_workspace_bytes(p, block, sigma_low, radius_low)
    if need == 0:
        st = lib().flr_denoise_lowres(ctypes.byref(p), block, sigma_low, radius_low, None, None,
                                      None, None, 0, None)
        check(st, "flr_denoise_lowres")
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=guides.device)
    if out is None:
        out = torch.empty((C, H, W), dtype=torch.float32, device=guides.device)
    _need(out, "out")
    check(lib().flr_denoise_lowres(ctypes.byref(p), block, sigma_low, radius_low,
                                   guides.data_ptr(), noisy.data_ptr(), out.data_ptr(),
                                   workspace.data_ptr(),
                                   workspace.numel() * workspace.element_size(),
                                   _stream(guides)), "flr_denoise_lowres")
    return out


# --------------------------------------------------------------------------
# Batched serving (flr_batch_plan / flr_batch_run)


class Batch:
    """Frames of uneven size through the two-pass path: one persistent
    launch over a work queue of every frame's tiles (``persistent_blocks``
    workgroups; 0 = one launch per stage). ``frames``: dicts with ``guides``
    [Q,H,W] and ``noisy`` [C,h,w] (h, w = H, W, or H/up, W/up for a joint
    frame, which then also gives ``guides_low`` [Q,h,w]); optional ``out``
    [C,H,W], ``tile_rows`` and ``apply_rows``. ``run()`` only launches kernels
    (graph-capturable); the plan and its workspace stay with the object."""

    def __init__(self, frames, radius: int = 8, eps: float = 1e-3, mode: str = "ridge",
                 eps_mul: float = 0.0, persistent_blocks: int | None = None):
        if not 1 <= len(frames) <= FLR_BATCH_MAX:
            raise ValueError(f"1..{FLR_BATCH_MAX} frames")
        Q = frames[0]["guides"].shape[0]
        C = frames[0]["noisy"].shape[0]
        dev = frames[0]["guides"].device
        self._keep = []
        arr = (FlrFrame * len(frames))()
        self.outs = []
        for i, f in enumerate(frames):
            g, y = f["guides"], f["noisy"]
            _need(g, "guides")
            _need(y, "noisy")
            low = f.get("guides_low")
            if low is not None:
                _need(low, "guides_low")
            if g.shape[0] != Q or y.shape[0] != C:
                raise ValueError("every frame needs the same guide and channel counts")
            out = f.get("out")
            if out is None:
                out = torch.empty((C,) + tuple(g.shape[1:]), dtype=torch.float32, device=dev)
            _need(out, "out")
            self.outs.append(out)
            self._keep += [g, y, out] + ([low] if low is not None else [])
            arr[i] = FlrFrame(height=g.shape[1], width=g.shape[2], noisy_height=y.shape[1],
                              noisy_width=y.shape[2], tile_rows=int(f.get("tile_rows", 0)),
                              apply_rows=int(f.get("apply_rows", 0)),
                              guides=g.data_ptr(),
                              guides_low=low.data_ptr() if low is not None else None,
                              noisy=y.data_ptr(), out=out.data_ptr())
        self.params = make_params(1, 1, Q, C, radius, eps=eps, mode=mode, eps_mul=eps_mul,
                                  average=True, fused="two_pass")
        self._frames = arr
        need = int(lib().flr_batch_workspace_bytes(ctypes.byref(self.params), arr, len(frames)))
        if need == 0:
            check(lib().flr_batch_plan(ctypes.byref(self.params), arr, len(frames), None, 0,
                                       None), "flr_batch_plan")
        self.workspace = torch.empty(need, dtype=torch.uint8, device=dev)
        self.plan = FlrBatch()
        check(lib().flr_batch_plan(ctypes.byref(self.params), arr, len(frames),
                                   self.workspace.data_ptr(), need, ctypes.byref(self.plan)),
              "flr_batch_plan")
        if persistent_blocks is not None:
            self.plan.persistent_blocks = int(persistent_blocks)
        self.device = dev

    def failed(self) -> bool:
        """Whether a persistent run gave up waiting (synchronises first)."""
        torch.cuda.synchronize(self.device)
        flag = ctypes.c_int32(0)
        check(lib().flr_batch_failed(ctypes.byref(self.plan), ctypes.byref(flag)),
              "flr_batch_failed")
        return bool(flag.value)

    def run(self):
        check(lib().flr_batch_run(ctypes.byref(self.plan),
                                  ctypes.c_void_p(torch.cuda.current_stream(self.device)
                                                  .cuda_stream)), "flr_batch_run")
        return self.outs


# --------------------------------------------------------------------------
# Adjoint (flr_denoise_backward) and autograd


def backward_workspace_bytes(p: FlrParams) -> int:
    return int(lib().flr_denoise_backward_workspace_bytes(ctypes.byref(p)))


def denoise_backward(noisy: torch.Tensor, guides: torch.Tensor, grad_out: torch.Tensor,
                     radius: int = 8, eps: float = 1e-3, mode: str = "ridge",
                     eps_mul: float = 0.0, average: bool = True,
                     workspace: torch.Tensor | None = None,
                     grad_noisy: torch.Tensor | None = None,
                     grad_guides: torch.Tensor | None = None,
                     grad_reg: torch.Tensor | None = None,
                     eps_device: torch.Tensor | None = None):
    """Gradients of ``denoise`` for dL/d(out) = ``grad_out`` [C,H,W]:
    (dL/d(noisy) [C,H,W], dL/d(guides) [Q,H,W], [dL/d(eps), dL/d(eps_mul)]
    as a float64 device tensor of 2). Moments are recomputed; the forward
    call's results are not needed. ``eps_device``: see make_params."""
    _need(guides, "guides")
    _need(noisy, "noisy")
    _need(grad_out, "grad_out")
    Q, H, W = guides.shape
    C = noisy.shape[0]
    if noisy.shape[1:] != guides.shape[1:] or grad_out.shape != noisy.shape:
        raise ValueError("noisy, guides and grad_out must share height and width; "
                         "grad_out must have the shape of noisy")
    p = make_params(H, W, Q, C, radius, eps=eps, mode=mode, eps_mul=eps_mul, average=average,
                    eps_device=eps_device)
    check(lib().flr_validate_params(ctypes.byref(p)), "flr_denoise_backward")
    need = backward_workspace_bytes(p)
    dev = guides.device
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    if grad_noisy is None:
        grad_noisy = torch.empty((C, H, W), dtype=torch.float32, device=dev)
    if grad_guides is None:
        grad_guides = torch.empty((Q, H, W), dtype=torch.float32, device=dev)
    if grad_reg is None:
        grad_reg = torch.empty(2, dtype=torch.float64, device=dev)
    _need(grad_noisy, "grad_noisy")
    _need(grad_guides, "grad_guides")
    if grad_reg.dtype != torch.float64 or grad_reg.numel() < 2 or grad_reg.device.type != "cuda":
        raise ValueError("grad_reg must be a float64 device tensor of at least 2 elements")
    check(lib().flr_denoise_backward(
        ctypes.byref(p), guides.data_ptr(), noisy.data_ptr(), grad_out.data_ptr(),
        grad_guides.data_ptr(), grad_noisy.data_ptr(), grad_reg.data_ptr(),
        workspace.data_ptr(), workspace.numel() * workspace.element_size(), _stream(guides)),
        "flr_denoise_backward")
    return grad_noisy, grad_guides, grad_reg


class _FLRFunction(torch.autograd.Function):
    """out = denoise(noisy, guides, ...) with its gradients from
    flr_denoise_backward. Saves only the inputs; the backward recomputes the
    window moments."""

    @staticmethod
    def forward(ctx, noisy, guides, eps, eps_mul, radius, mode, average, fused):
        e = float(eps)
        m = float(eps_mul)
        ctx.cfg = (radius, e, mode, m, average)
        ctx.save_for_backward(noisy, guides)
        return denoise(noisy, guides, radius=radius, eps=e, mode=mode, eps_mul=m,
                       average=average, fused=fused)

    @staticmethod
    def backward(ctx, grad_out):
        noisy, guides = ctx.saved_tensors
        radius, e, mode, m, average = ctx.cfg
        gy, gg, gr = denoise_backward(noisy, guides, grad_out.contiguous().float(), radius, e,
                                      mode, m, average)
        need = ctx.needs_input_grad
        ge = gr[0].float() if need[2] else None
        gm = gr[1].float() if need[3] else None
        return (gy if need[0] else None, gg if need[1] else None, ge, gm, None, None, None, None)


def flr(noisy: torch.Tensor, guides: torch.Tensor, radius: int = 8, eps=1e-3,
        mode: str = "ridge", eps_mul=0.0, average: bool = True, fused="two_pass") -> torch.Tensor:
    """Differentiable FLR: ``denoise`` under torch autograd. ``eps`` and
    ``eps_mul`` may be 0-d tensors that require grad (their values are read
    on the host each call); gradients reach noisy, guides and both."""
    if not torch.is_tensor(eps):
        eps = torch.tensor(float(eps), dtype=torch.float32)
    if not torch.is_tensor(eps_mul):
        eps_mul = torch.tensor(float(eps_mul), dtype=torch.float32)
    return _FLRFunction.apply(noisy, guides, eps, eps_mul, radius, mode, average, fused)


# --------------------------------------------------------------------------
# FLNR guide network (include/flr_net.h)

NET_IN_GUIDES, NET_IN_NOISY, NET_OUT = 8, 3, 4


def net_num_params() -> int:
    return int(lib().flr_net_num_params())


def net_pack(params: torch.Tensor) -> torch.Tensor:
    """FP32 parameter vector (layer order of include/flr_net.h) -> the packed
    BF16 device block (uint8 tensor) that net_forward and flnr_denoise read."""
    _need(params, "params", ndim=1)
    if params.numel() != net_num_params():
        raise ValueError(f"expected {net_num_params()} parameters, got {params.numel()}")
    packed = torch.empty(int(lib().flr_net_packed_bytes()), dtype=torch.uint8,
                         device=params.device)
    check(lib().flr_net_pack(params.data_ptr(), packed.data_ptr(), _stream(params)),
          "flr_net_pack")
    return packed


def net_forward(guides: torch.Tensor, noisy: torch.Tensor, packed: torch.Tensor,
                out: torch.Tensor | None = None,
                workspace: torch.Tensor | None = None) -> torch.Tensor:
    """The 4 extra guide planes [4,H,W] for guides [8,H,W] and noisy [3,H,W]."""
    _need(guides, "guides")
    _need(noisy, "noisy")
    if guides.shape[0] != NET_IN_GUIDES or noisy.shape[0] != NET_IN_NOISY:
        raise ValueError("the network reads 8 guide planes and 3 noisy planes")
    _, H, W = guides.shape
    need = int(lib().flr_net_workspace_bytes(H, W))
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=guides.device)
    if out is None:
        out = torch.empty((NET_OUT, H, W), dtype=torch.float32, device=guides.device)
    _need(out, "out")
    check(lib().flr_net_forward(H, W, guides.data_ptr(), noisy.data_ptr(), packed.data_ptr(),
                                out.data_ptr(), workspace.data_ptr(),
                                workspace.numel() * workspace.element_size(), _stream(guides)),
          "flr_net_forward")
    return out


# names of the trace tensors of net_forward_trace, in index order
NET_TRACE_NAMES = ("x0", "in3", "in1", "e1a", "e1b", "e2a", "e2b", "d1a", "d1b", "d0a", "d0b",
                   "out3")


def net_trace_layout(H: int, W: int) -> dict:
    """name -> (byte offset, channels, height, width) of each trace tensor."""
    out = {}
    for i, name in enumerate(NET_TRACE_NAMES):
        off = ctypes.c_size_t()
        c, h, w = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().flr_net_trace_tensor(H, W, i, ctypes.byref(off), ctypes.byref(c),
                                         ctypes.byref(h), ctypes.byref(w)),
              "flr_net_trace_tensor")
        out[name] = (off.value, c.value, h.value, w.value)
    return out


def net_forward_trace(guides: torch.Tensor, noisy: torch.Tensor, packed: torch.Tensor):
    """net_forward, also returning every layer's BF16 output activation:
    (out [4,H,W] float32, {name: int16 tensor [h, w, channels] of BF16 bit
    patterns}) with the names of NET_TRACE_NAMES."""
    _need(guides, "guides")
    _need(noisy, "noisy")
    if guides.shape[0] != NET_IN_GUIDES or noisy.shape[0] != NET_IN_NOISY:
        raise ValueError("the network reads 8 guide planes and 3 noisy planes")
    _, H, W = guides.shape
    need = int(lib().flr_net_trace_bytes(H, W))
    trace = torch.empty(max(need, 1), dtype=torch.uint8, device=guides.device)
    out = torch.empty((NET_OUT, H, W), dtype=torch.float32, device=guides.device)
    check(lib().flr_net_forward_trace(H, W, guides.data_ptr(), noisy.data_ptr(),
                                      packed.data_ptr(), out.data_ptr(), trace.data_ptr(), need,
                                      _stream(guides)),
          "flr_net_forward_trace")
    acts = {}
    for name, (off, c, h, w) in net_trace_layout(H, W).items():
        acts[name] = trace[off:off + h * w * c * 2].view(torch.int16).view(h, w, c)
    return out, acts


def net_backward(guides: torch.Tensor, noisy: torch.Tensor, params: torch.Tensor,
                 packed: torch.Tensor, grad_out: torch.Tensor,
                 grad_params: torch.Tensor | None = None, accumulate: bool = False,
                 workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Gradient of a loss with respect to the FP32 parameters ``params``
    (packed = net_pack(params)) given its gradient ``grad_out`` [4,H,W] with
    respect to net_forward's output. accumulate=True adds into grad_params."""
    _need(guides, "guides")
    _need(noisy, "noisy")
    _need(grad_out, "grad_out")
    _need(params, "params", ndim=1)
    if guides.shape[0] != NET_IN_GUIDES or noisy.shape[0] != NET_IN_NOISY or \
            grad_out.shape[0] != NET_OUT:
        raise ValueError("the network reads 8 guide and 3 noisy planes and writes 4")
    _, H, W = guides.shape
    need = int(lib().flr_net_backward_workspace_bytes(H, W))
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=guides.device)
    if grad_params is None:
        if accumulate:
            raise ValueError("accumulate needs grad_params")
        grad_params = torch.empty_like(params)
    _need(grad_params, "grad_params", ndim=1)
    check(lib().flr_net_backward(H, W, guides.data_ptr(), noisy.data_ptr(), params.data_ptr(),
                                 packed.data_ptr(), grad_out.data_ptr(), grad_params.data_ptr(),
                                 int(bool(accumulate)), workspace.data_ptr(),
                                 workspace.numel() * workspace.element_size(), _stream(guides)),
          "flr_net_backward")
    return grad_params


def flnr_workspace_bytes(p: FlrParams) -> int:
    return int(lib().flr_flnr_workspace_bytes(ctypes.byref(p)))


def flnr_denoise(noisy: torch.Tensor, guides12: torch.Tensor, packed: torch.Tensor,
                 radius: int = 8, eps: float = 1e-3, mode: str = "ridge", eps_mul: float = 0.0,
                 average: bool = True, fused="two_pass", out: torch.Tensor | None = None,
                 workspace: torch.Tensor | None = None) -> torch.Tensor:
    """FLNR: guides12 [12,H,W] holds the 8 input guides in planes 0..7; the
    network writes planes 8..11, then FLR runs over all 12 -> [3,H,W]."""
    _need(guides12, "guides12")
    _need(noisy, "noisy")
    Q, H, W = guides12.shape
    C = noisy.shape[0]
    p = make_params(H, W, Q, C, radius, eps=eps, mode=mode, eps_mul=eps_mul, average=average,
                    fused=fused)
    need = flnr_workspace_bytes(p)
    if need == 0:
        check(lib().flr_validate_params(ctypes.byref(p)), "flr_flnr_denoise")
        raise ValueError("FLNR needs 12 guide planes and 3 noisy channels")
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=guides12.device)
    if out is None:
        out = torch.empty((C, H, W), dtype=torch.float32, device=guides12.device)
    _need(out, "out")
    check(lib().flr_flnr_denoise(ctypes.byref(p), guides12.data_ptr(), noisy.data_ptr(),
                                 packed.data_ptr(), out.data_ptr(), workspace.data_ptr(),
                                 workspace.numel() * workspace.element_size(), _stream(guides12)),
          "flr_flnr_denoise")
    return out


# Training step (include/flr_train.h)

def l1_loss_grad(out: torch.Tensor, target: torch.Tensor, scale: float,
                 grad: torch.Tensor | None = None, loss: torch.Tensor | None = None,
                 workspace: torch.Tensor | None = None):
    """(grad, loss): grad = scale sign(out - target) (shape of out), loss a
    float64 device tensor of one element, scale * sum |out - target|."""
    for t, name in ((out, "out"), (target, "target")):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or \
                t.device.type != "cuda" or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 device tensor")
    if out.shape != target.shape:
        raise ValueError("out and target must have the same shape")
    n = out.numel()
    if grad is None:
        grad = torch.empty_like(out)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device=out.device)
    need = int(lib().flr_l1_workspace_bytes(n))
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=out.device)
    check(lib().flr_l1_loss_grad(n, out.data_ptr(), target.data_ptr(), float(scale),
                                 grad.data_ptr(), loss.data_ptr(), workspace.data_ptr(),
                                 workspace.numel(), _stream(out)), "flr_l1_loss_grad")
    return grad, loss


def adamw_step(params: torch.Tensor, grads: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
               step: int, lr: float, betas=(0.9, 0.999), eps: float = 1e-8,
               weight_decay: float = 0.0) -> None:
    """AdamW update of params (in place) with moments m, v (in place)."""
    for t, name in ((params, "params"), (grads, "grads"), (m, "m"), (v, "v")):
        _need(t, name, ndim=1)
        if t.numel() != params.numel():
            raise ValueError(f"{name} must have {params.numel()} elements")
    check(lib().flr_adamw_step(params.numel(), params.data_ptr(), grads.data_ptr(), m.data_ptr(),
                               v.data_ptr(), int(step), float(lr), float(betas[0]),
                               float(betas[1]), float(eps), float(weight_decay),
                               _stream(params)), "flr_adamw_step")


def reg_adam_step(reg: torch.Tensor, state: torch.Tensor, dreg: torch.Tensor, lr: float,
                  betas=(0.9, 0.999), adam_eps: float = 1e-12, learn_mul: bool = False) -> None:
    """Adam on log eps (and log eps_mul) on the device: ``reg`` float32 (2),
    ``state`` float64 (6, zeros before the first step), ``dreg`` float64
    [n, 2] per-crop regulariser gradients; reg and state in place."""
    for t, dt, n, name in ((reg, torch.float32, 2, "reg"), (state, torch.float64, 6, "state")):
        if not isinstance(t, torch.Tensor) or t.dtype != dt or t.device.type != "cuda" or \
                t.numel() != n or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dt} device tensor of {n}")
    if dreg.dtype != torch.float64 or dreg.device.type != "cuda" or not dreg.is_contiguous() or \
            dreg.numel() % 2:
        raise ValueError("dreg must be a contiguous float64 device tensor [n, 2]")
    check(lib().flr_reg_adam_step(reg.data_ptr(), state.data_ptr(), dreg.data_ptr(),
                                  dreg.numel() // 2, float(lr), float(betas[0]), float(betas[1]),
                                  float(adam_eps), int(bool(learn_mul)), _stream(reg)),
          "flr_reg_adam_step")


class FLNRTrainer:
    """Training of the guide network through FLR (Sec. 3.3): per crop the
    network writes guide planes 8..11, FLR (two-pass path) denoises over the
    12 guides, the L1 loss against the target gives dL/d(out), the FLR adjoint
    gives dL/d(guides) and the network backward accumulates dL/d(weights);
    then one AdamW step updates the FP32 master weights. ``params`` (FP32
    device vector) is updated in place. Buffers are allocated once per crop
    size and reused.

    FLR's regularisers live on the device (``reg``: eps, eps_mul) and every
    FLR call reads them from there. With ``learn_eps`` they are learned with
    the network, as the Appendix learns its regularisers by backpropagation:
    Adam on their logarithms from the adjoint's gradients summed over the
    batch, in a device kernel with its own step count (no host read per
    step); ``mode="paper"`` with ``flr_eps_mul > 0`` learns eps_mul too."""

    def __init__(self, params: torch.Tensor, lr: float = 1e-3, betas=(0.9, 0.999),
                 eps: float = 1e-8, weight_decay: float = 0.0, radius: int = 8,
                 flr_eps: float = 1e-3, learn_eps: bool = False, eps_lr: float = 1e-2,
                 mode: str = "ridge", flr_eps_mul: float = 0.0):
        _need(params, "params", ndim=1)
        if params.numel() != net_num_params():
            raise ValueError(f"expected {net_num_params()} parameters")
        if mode not in _MODES:
            raise ValueError(f"mode must be one of {sorted(_MODES)}")
        self.params = params
        dev = params.device
        self.grad = torch.zeros_like(params)
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.t = 0
        self.lr, self.betas, self.eps, self.wd = lr, betas, eps, weight_decay
        self.radius, self.mode = radius, mode
        self.reg = torch.tensor([flr_eps, flr_eps_mul], dtype=torch.float32, device=dev)
        self.reg_state = torch.zeros(6, dtype=torch.float64, device=dev)
        self.learn_eps, self.eps_lr = learn_eps, eps_lr
        self.last_dreg = None
        self._bufs = {}

    @property
    def flr_eps(self) -> float:
        """The current eps of FLR (a host read of the device value)."""
        return float(self.reg[0].item())

    @property
    def flr_eps_mul(self) -> float:
        return float(self.reg[1].item())

    def state_dict(self) -> dict:
        """Checkpoint: the FP32 master weights, the AdamW moments and step
        count, FLR's regularisers with their optimizer state, and the
        hyperparameters (tensors copied to the host)."""
        return {"params": self.params.detach().cpu().clone(), "m": self.m.cpu().clone(),
                "v": self.v.cpu().clone(), "step": int(self.t), "lr": self.lr,
                "betas": tuple(self.betas), "eps": self.eps, "weight_decay": self.wd,
                "radius": self.radius, "mode": self.mode, "reg": self.reg.cpu().clone(),
                "reg_state": self.reg_state.cpu().clone(), "learn_eps": self.learn_eps,
                "eps_lr": self.eps_lr}

    def load_state_dict(self, state: dict) -> None:
        """Resume from state_dict(): the next step equals the one the saved
        trainer would have taken."""
        for k in ("params", "m", "v"):
            if state[k].numel() != self.params.numel():
                raise ValueError(f"checkpoint {k} has {state[k].numel()} elements, "
                                 f"expected {self.params.numel()}")
        self.params.copy_(state["params"])
        self.m.copy_(state["m"])
        self.v.copy_(state["v"])
        self.t = int(state["step"])
        self.lr, self.betas, self.eps, self.wd = (state["lr"], tuple(state["betas"]),
                                                  state["eps"], state["weight_decay"])
        self.radius = state["radius"]
        self.mode = state.get("mode", "ridge")
        if "reg" in state:
            self.reg.copy_(state["reg"])
            self.reg_state.copy_(state["reg_state"])
        else:  # a checkpoint that kept eps on the host
            self.reg.copy_(torch.tensor([state["flr_eps"], 0.0]))
            self.reg_state.zero_()
        self.learn_eps = state.get("learn_eps", False)
        self.eps_lr = state.get("eps_lr", self.eps_lr)

    def _buffers(self, H, W, dev):
        key = (H, W)
        if key not in self._bufs:
            p = make_params(H, W, 12, 3, self.radius, mode=self.mode, fused="two_pass")
            b = dict(
                g12=torch.empty((12, H, W), dtype=torch.float32, device=dev),
                out=torch.empty((3, H, W), dtype=torch.float32, device=dev),
                G=torch.empty((3, H, W), dtype=torch.float32, device=dev),
                dy=torch.empty((3, H, W), dtype=torch.float32, device=dev),
                dg=torch.empty((12, H, W), dtype=torch.float32, device=dev),
                ws_fwd=torch.empty(max(workspace_bytes(p), 1), dtype=torch.uint8, device=dev),
                ws_bwd=torch.empty(max(backward_workspace_bytes(p), 1), dtype=torch.uint8,
                                   device=dev),
                ws_net=torch.empty(max(int(lib().flr_net_backward_workspace_bytes(H, W)), 1),
                                   dtype=torch.uint8, device=dev),
                ws_l1=torch.empty(max(int(lib().flr_l1_workspace_bytes(3 * H * W)), 1),
                                  dtype=torch.uint8, device=dev))
            self._bufs[key] = b
        return self._bufs[key]

    def step(self, crops) -> torch.Tensor:
        """One step on a batch: crops is a list of dicts with device tensors
        ``guides`` [8,H,W] (or ``guides12`` [12,H,W] with the 8 guides in
        planes 0..7; the network overwrites 8..11), ``noisy`` and ``target``
        [3,H,W]. Returns the per-crop losses (float64 device tensor; their
        sum is the batch mean absolute error). Nothing is read back to the
        host."""
        dev = self.params.device
        packed = net_pack(self.params)
        losses = torch.empty(len(crops), dtype=torch.float64, device=dev)
        dregs = torch.empty((len(crops), 2), dtype=torch.float64, device=dev)
        total = sum(c["noisy"].numel() for c in crops)
        for k, c in enumerate(crops):
            _, H, W = c["noisy"].shape
            b = self._buffers(H, W, dev)
            if "guides12" in c:  # the caller's 12-plane buffer, planes 0..7 filled
                g12 = c["guides12"]
            else:
                g12 = b["g12"]
                g12[:NET_IN_GUIDES].copy_(c["guides"])
            net_forward(g12[:NET_IN_GUIDES], c["noisy"], packed, out=g12[NET_IN_GUIDES:],
                        workspace=b["ws_net"])
            denoise(c["noisy"], g12, self.radius, mode=self.mode, fused="two_pass",
                    out=b["out"], workspace=b["ws_fwd"], eps_device=self.reg)
            l1_loss_grad(b["out"], c["target"], 1.0 / total, grad=b["G"], loss=losses[k:k + 1],
                         workspace=b["ws_l1"])
            denoise_backward(c["noisy"], g12, b["G"], self.radius, mode=self.mode,
                             workspace=b["ws_bwd"], grad_noisy=b["dy"], grad_guides=b["dg"],
                             grad_reg=dregs[k], eps_device=self.reg)
            net_backward(g12[:NET_IN_GUIDES], c["noisy"], self.params, packed,
                         b["dg"][NET_IN_GUIDES:], grad_params=self.grad, accumulate=k > 0,
                         workspace=b["ws_net"])
        self.t += 1
        adamw_step(self.params, self.grad, self.m, self.v, self.t, self.lr, self.betas, self.eps,
                   self.wd)
        self.last_dreg = dregs
        if self.learn_eps:
            reg_adam_step(self.reg, self.reg_state, dregs, self.eps_lr, self.betas,
                          learn_mul=self.mode == "paper")
        return losses


__all__ = ["FLRError", "PATHS", "make_params", "num_moment_planes", "num_coeff_planes",
           "workspace_bytes", "moments", "solve", "coefficients", "apply", "denoise",
           "net_num_params", "net_pack", "net_forward", "net_backward", "flnr_workspace_bytes",
           "flnr_denoise", "l1_loss_grad", "adamw_step", "reg_adam_step", "FLNRTrainer"]
