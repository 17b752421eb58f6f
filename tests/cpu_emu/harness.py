"""Build and drive the host-executed build of the FLR kernel sources.

``build()`` compiles ``emu.cpp`` (the kernel templates) and the library's
own ``flr_api.cpp`` with g++ into ``_build/libflr_emu.so``; ``Emu`` calls the
real C ABI entry points on guard-paged host buffers. Run as a script it
executes one named case and prints a JSON line, so that a crash in the
emulated kernels cannot take down the test runner. Test infrastructure only.
"""
from __future__ import annotations

import ctypes
import fcntl
import json
import os
import subprocess
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2410_11625_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
# Optional numeric-policy override, e.g. "FLR_SUM_T=double,FLR_SOLVE_T=double"
# (used to compare precision variants of the same sources).
VARIANT = os.environ.get("FLR_EMU_VARIANT", "")
# FLR_EMU_SANITIZE=1: AddressSanitizer + UndefinedBehaviorSanitizer build of
# the same sources (host code only: the kernels run on the host here), with
# the ROCm LLVM clang++ as host compiler (GCC 11's UBSan instrumentation of
# these sources gives wrong results without a report; clang's is clean); the
# process that loads it needs the ASan runtime preloaded (sanitizer_env()).
SANITIZE = os.environ.get("FLR_EMU_SANITIZE", "") == "1"
SAN_CXX = "/opt/rocm/llvm/bin/clang++"
SO = os.path.join(BUILD, "libflr_emu%s%s.so" % (
    "_" + VARIANT.replace("=", "-").replace(",", "_") if VARIANT else "",
    "_asan_ubsan" if SANITIZE else ""))
# FLR_EMU_EXTRA: further compiler flags for a one-off build (named in the .so)
EXTRA = os.environ.get("FLR_EMU_EXTRA", "").split()
if EXTRA:
    SO = SO[:-3] + "_x%08x.so" % (hash(" ".join(EXTRA)) & 0xffffffff)
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-shared-libsan", "-fno-omit-frame-pointer"]

sys.path.insert(0, ROOT)
from paper_2410_11625_amd._lib import FlrParams  # noqa: E402  (ctypes struct layout only)


def sanitizer_env() -> dict:
    """Environment of a subprocess that loads the sanitizer build: the ASan
    runtime preloaded into the (uninstrumented) Python process, leak
    checking off (the interpreter's own allocations), every report fatal."""
    asan = subprocess.run([SAN_CXX, "-print-file-name=libclang_rt.asan-x86_64.so"],
                          stdout=subprocess.PIPE, text=True, check=True).stdout.strip()
    if not os.path.isabs(asan):
        import glob
        asan = sorted(glob.glob(os.path.join(os.path.dirname(os.path.dirname(SAN_CXX)), "lib",
                                             "clang", "*", "lib", "linux",
                                             "libclang_rt.asan-x86_64.so")))[-1]
    env = dict(os.environ)
    env["FLR_EMU_SANITIZE"] = "1"
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = ("detect_leaks=0:abort_on_error=1:detect_stack_use_after_return=0:"
                           "clear_shadow_mmap_threshold=1048576")
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    return env


def build(force: bool = False) -> str:
    srcs = [os.path.join(HERE, "emu.cpp"), os.path.join(CSRC, "flr_api.cpp")]
    net_src = os.path.join(CSRC, "flr_net.hip")
    adj_src = os.path.join(CSRC, "flr_adjoint.hip")
    lr_src = os.path.join(CSRC, "flr_lowres.hip")
    deps = srcs + [net_src, adj_src, lr_src, os.path.join(HERE, "hip", "hip_runtime.h"),
                   os.path.join(CSRC, "flr_device.hpp"), os.path.join(CSRC, "flr_launch.hpp"),
                   os.path.join(CSRC, "flr_adjoint.hpp"), os.path.join(CSRC, "flr_lowres.hpp"),
                   os.path.join(CSRC, "flr_net_bwd.hpp"), os.path.join(CSRC, "flr_box.hpp"),
                   os.path.join(CSRC, "flr_prefix.hpp"),
                   os.path.join(INCLUDE, "flr.h"), os.path.join(INCLUDE, "flr_net.h")]
    def fresh():
        return os.path.exists(SO) and \
            os.path.getmtime(SO) >= max(os.path.getmtime(d) for d in deps)

    if not force and fresh():
        return SO
    os.makedirs(BUILD, exist_ok=True)
    # one builder at a time (test workers may ask concurrently)
    with open(SO + ".lock", "w") as lk:
        fcntl.flock(lk, fcntl.LOCK_EX)
        if not force and fresh():
            return SO
        defs = [f"-D{d}" for d in VARIANT.split(",") if d]
        tmp = f"{SO}.tmp{os.getpid()}"
        cxx = SAN_CXX if SANITIZE else os.environ.get("FLR_EMU_CXX", "g++")
        tls = [] if "clang" in os.path.basename(cxx) else ["-fno-extern-tls-init"]
        # the sanitizer build compiles unoptimised (minutes faster to build;
        # its cases are small)
        opt = ["-O0", "-g1"] if SANITIZE else ["-O1", "-g"]
        flags = [cxx, "-std=c++20", *opt, "-pthread", *tls, "-fPIC", *defs,
                 *(SAN_FLAGS if SANITIZE else []), *EXTRA, f"-I{HERE}", f"-I{INCLUDE}",
                 f"-I{CSRC}"]
        units = srcs + [net_src, adj_src, lr_src]
        objs = [f"{tmp}.{i}.o" for i in range(len(units))]

        def compile_unit(i):
            subprocess.run([*flags, "-x", "c++", "-c", units[i], "-o", objs[i]], check=True)

        import concurrent.futures as cf
        with cf.ThreadPoolExecutor(max_workers=len(units)) as ex:
            list(ex.map(compile_unit, range(len(units))))
        link = [cxx, "-shared", "-pthread", *(SAN_FLAGS if SANITIZE else []), *objs, "-o", tmp]
        subprocess.run(link, check=True)
        for o in objs:
            os.remove(o)
        os.replace(tmp, SO)
    return SO


class Emu:
    def __init__(self):
        L = ctypes.CDLL(build())
        vp = ctypes.c_void_p
        P = ctypes.POINTER(FlrParams)
        L.emu_alloc.argtypes = [ctypes.c_size_t]
        L.emu_alloc.restype = vp
        L.emu_free.argtypes = [vp, ctypes.c_size_t]
        L.emu_message.restype = ctypes.c_char_p
        L.flr_moments.argtypes = [P, vp, vp, vp, vp]
        L.flr_solve.argtypes = [P, vp, vp, vp]
        L.flr_apply.argtypes = [P, vp, vp, vp, vp]
        L.flr_denoise.argtypes = [P, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.flr_denoise_workspace_bytes.argtypes = [P]
        L.flr_denoise_workspace_bytes.restype = ctypes.c_size_t
        L.flr_num_moment_planes.restype = ctypes.c_size_t
        L.flr_num_coeff_planes.restype = ctypes.c_size_t
        self.L = L
        self._bufs = []

    def buf(self, arr=None, shape=None):
        """Guard-paged float32 buffer (copy of ``arr`` or uninitialised NaNs)."""
        if arr is not None:
            arr = np.ascontiguousarray(arr, dtype=np.float32)
            shape = arr.shape
        nbytes = int(np.prod(shape)) * 4
        ptr = self.L.emu_alloc(max(nbytes, 4))
        view = np.ctypeslib.as_array((ctypes.c_float * max(nbytes // 4, 1)).from_address(ptr))
        view = view[: nbytes // 4].reshape(shape)
        if arr is not None:
            view[...] = arr
        else:
            view[...] = np.nan
        self._bufs.append((ptr, nbytes))
        return ptr, view

    def close(self):
        for ptr, n in self._bufs:
            self.L.emu_free(ptr, max(n, 4))
        self._bufs = []

    def check(self, st, what):
        if st != 0:
            raise RuntimeError(f"{what} returned {st}: {self.L.emu_message().decode()}")

    def denoise(self, noisy, guides, p: FlrParams):
        gp, _ = self.buf(guides)
        yp, _ = self.buf(noisy)
        op, out = self.buf(shape=noisy.shape)
        need = self.L.flr_denoise_workspace_bytes(ctypes.byref(p))
        wp = self.buf(shape=(max(need // 4, 1),))[0] if need else None
        self.check(self.L.flr_denoise(ctypes.byref(p), gp, yp, op, wp, need, None), "flr_denoise")
        return out.copy()

    def net(self, guides, noisy, params):
        """The guide network: FP32 parameters -> packed, then forward -> [4,H,W]."""
        L = self.L
        vp = ctypes.c_void_p
        L.flr_net_num_params.restype = ctypes.c_size_t
        L.flr_net_packed_bytes.restype = ctypes.c_size_t
        L.flr_net_workspace_bytes.restype = ctypes.c_size_t
        L.flr_net_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.flr_net_pack.argtypes = [vp, vp, vp]
        L.flr_net_forward.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, vp,
                                      ctypes.c_size_t, vp]
        _, H, W = guides.shape
        pp, _ = self.buf(params)
        kb = int(L.flr_net_packed_bytes())
        kp, _ = self.buf(shape=(kb // 4,))
        self.check(L.flr_net_pack(pp, kp, None), "flr_net_pack")
        gp, _ = self.buf(guides)
        yp, _ = self.buf(noisy)
        op, out = self.buf(shape=(4, H, W))
        need = int(L.flr_net_workspace_bytes(H, W))
        wp, _ = self.buf(shape=(need // 4,))
        self.check(L.flr_net_forward(H, W, gp, yp, kp, op, wp, need, None), "flr_net_forward")
        return out.copy()

    def net_trace(self, guides, noisy, params):
        """flr_net_forward_trace -> (out [4,H,W], {name: HWC int16 BF16 tensor})."""
        L = self.L
        vp = ctypes.c_void_p
        i32 = ctypes.c_int32
        L.flr_net_packed_bytes.restype = ctypes.c_size_t
        L.flr_net_pack.argtypes = [vp, vp, vp]
        L.flr_net_trace_bytes.restype = ctypes.c_size_t
        L.flr_net_trace_bytes.argtypes = [i32, i32]
        L.flr_net_trace_tensor.argtypes = [i32, i32, i32, ctypes.POINTER(ctypes.c_size_t),
                                           ctypes.POINTER(i32), ctypes.POINTER(i32),
                                           ctypes.POINTER(i32)]
        L.flr_net_forward_trace.argtypes = [i32, i32, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        _, H, W = guides.shape
        pp, _ = self.buf(params)
        kb = int(L.flr_net_packed_bytes())
        kp, _ = self.buf(shape=(kb // 4,))
        self.check(L.flr_net_pack(pp, kp, None), "flr_net_pack")
        gp, _ = self.buf(guides)
        yp, _ = self.buf(noisy)
        op, out = self.buf(shape=(4, H, W))
        need = int(L.flr_net_trace_bytes(H, W))
        tp, tr = self.buf(shape=((need + 3) // 4,))
        self.check(L.flr_net_forward_trace(H, W, gp, yp, kp, op, tp, need, None),
                   "flr_net_forward_trace")
        raw = tr.view(np.uint8)
        names = ("x0", "in3", "in1", "e1a", "e1b", "e2a", "e2b", "d1a", "d1b", "d0a", "d0b",
                 "out3")
        acts = {}
        for i, name in enumerate(names):
            off, c, h, w = ctypes.c_size_t(), i32(), i32(), i32()
            self.check(L.flr_net_trace_tensor(H, W, i, ctypes.byref(off), ctypes.byref(c),
                                              ctypes.byref(h), ctypes.byref(w)),
                       "flr_net_trace_tensor")
            n = h.value * w.value * c.value * 2
            acts[name] = raw[off.value:off.value + n].view(np.int16).reshape(
                h.value, w.value, c.value).copy()
        return out.copy(), acts

    def net_backward(self, guides, noisy, params, grad_out):
        """flr_net_backward -> FP32 parameter gradients (layout of params)."""
        L = self.L
        vp = ctypes.c_void_p
        L.flr_net_packed_bytes.restype = ctypes.c_size_t
        L.flr_net_pack.argtypes = [vp, vp, vp]
        L.flr_net_backward_workspace_bytes.restype = ctypes.c_size_t
        L.flr_net_backward_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.flr_net_backward.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, vp, vp,
                                       ctypes.c_int32, vp, ctypes.c_size_t, vp]
        _, H, W = guides.shape
        pp, _ = self.buf(params)
        kb = int(L.flr_net_packed_bytes())
        kp, _ = self.buf(shape=(kb // 4,))
        self.check(L.flr_net_pack(pp, kp, None), "flr_net_pack")
        gp, _ = self.buf(guides)
        yp, _ = self.buf(noisy)
        dp, _ = self.buf(grad_out)
        op, out = self.buf(shape=params.shape)
        need = int(L.flr_net_backward_workspace_bytes(H, W))
        wp, _ = self.buf(shape=(need // 4,))
        self.check(L.flr_net_backward(H, W, gp, yp, pp, kp, dp, op, 0, wp, need, None),
                   "flr_net_backward")
        return out.copy()

    def backward(self, noisy, guides, grad_out, p: FlrParams):
        """flr_denoise_backward -> (d_noisy, d_guides, [d_eps, d_eps_mul])."""
        L = self.L
        vp = ctypes.c_void_p
        L.flr_denoise_backward_workspace_bytes.argtypes = [ctypes.POINTER(FlrParams)]
        L.flr_denoise_backward_workspace_bytes.restype = ctypes.c_size_t
        L.flr_denoise_backward.argtypes = [ctypes.POINTER(FlrParams), vp, vp, vp, vp, vp, vp, vp,
                                           ctypes.c_size_t, vp]
        gp, _ = self.buf(guides)
        yp, _ = self.buf(noisy)
        op, _ = self.buf(grad_out)
        dgp, dg = self.buf(shape=guides.shape)
        dyp, dy = self.buf(shape=noisy.shape)
        rp, reg = self.buf(shape=(4,))
        need = int(L.flr_denoise_backward_workspace_bytes(ctypes.byref(p)))
        wp, _ = self.buf(shape=(need // 4,))
        self.check(L.flr_denoise_backward(ctypes.byref(p), gp, yp, op, dgp, dyp, rp, wp, need,
                                          None), "flr_denoise_backward")
        return dy.copy(), dg.copy(), reg.copy().view(np.float64).copy()

    def lowres(self, noisy, guides, p: FlrParams, block, sigma, radius_low):
        """flr_denoise_lowres -> [C,H,W]."""
        L = self.L
        vp = ctypes.c_void_p
        P = ctypes.POINTER(FlrParams)
        L.flr_lowres_workspace_bytes.argtypes = [P, ctypes.c_int32, ctypes.c_float, ctypes.c_int32]
        L.flr_lowres_workspace_bytes.restype = ctypes.c_size_t
        L.flr_denoise_lowres.argtypes = [P, ctypes.c_int32, ctypes.c_float, ctypes.c_int32, vp, vp,
                                         vp, vp, ctypes.c_size_t, vp]
        gp, _ = self.buf(guides)
        yp, _ = self.buf(noisy)
        op, out = self.buf(shape=noisy.shape)
        need = int(L.flr_lowres_workspace_bytes(ctypes.byref(p), block, sigma, radius_low))
        wp, _ = self.buf(shape=(need // 4,))
        self.check(L.flr_denoise_lowres(ctypes.byref(p), block, sigma, radius_low, gp, yp, op, wp,
                                        need, None), "flr_denoise_lowres")
        return out.copy()

    def batch(self, frames, p: FlrParams, persistent_blocks=None, runs=1):
        """flr_batch_plan + flr_batch_run over frames (dicts of guides, noisy,
        optional guides_low) -> list of outputs (of the last of `runs` runs;
        with `persistent_blocks` set, the plan's persistent grid is replaced;
        0 runs one launch per stage). Also sets self.batch_failed."""
        from paper_2410_11625_amd._lib import FlrBatch, FlrFrame
        L = self.L
        F = ctypes.POINTER(FlrFrame)
        Bp = ctypes.POINTER(FlrBatch)
        P = ctypes.POINTER(FlrParams)
        L.flr_batch_workspace_bytes.argtypes = [P, F, ctypes.c_int32]
        L.flr_batch_workspace_bytes.restype = ctypes.c_size_t
        L.flr_batch_plan.argtypes = [P, F, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t, Bp]
        L.flr_batch_run.argtypes = [Bp, ctypes.c_void_p]
        arr = (FlrFrame * len(frames))()
        outs = []
        for i, f in enumerate(frames):
            gp, _ = self.buf(f["guides"])
            yp, _ = self.buf(f["noisy"])
            lp = self.buf(f["guides_low"])[0] if f.get("guides_low") is not None else None
            C = f["noisy"].shape[0]
            H, W = f["guides"].shape[1:]
            op, out = self.buf(shape=(C, H, W))
            outs.append(out)
            arr[i] = FlrFrame(height=H, width=W, noisy_height=f["noisy"].shape[1],
                              noisy_width=f["noisy"].shape[2], tile_rows=f.get("tile_rows", 0),
                              guides=gp, guides_low=lp, noisy=yp, out=op)
        need = int(L.flr_batch_workspace_bytes(ctypes.byref(p), arr, len(frames)))
        wp, _ = self.buf(shape=(need // 4,))
        plan = FlrBatch()
        self.check(L.flr_batch_plan(ctypes.byref(p), arr, len(frames), wp, need,
                                    ctypes.byref(plan)), "flr_batch_plan")
        if persistent_blocks is not None:
            plan.persistent_blocks = persistent_blocks
        for _ in range(runs):
            for o in outs:
                o[...] = np.nan
            self.check(L.flr_batch_run(ctypes.byref(plan), None), "flr_batch_run")
        L.flr_batch_failed.argtypes = [Bp, ctypes.POINTER(ctypes.c_int32)]
        flag = ctypes.c_int32(0)
        self.check(L.flr_batch_failed(ctypes.byref(plan), ctypes.byref(flag)), "flr_batch_failed")
        self.batch_failed = bool(flag.value)
        return [o.copy() for o in outs]

    def moments(self, noisy, guides, p: FlrParams):
        Q, H, W = guides.shape
        C = noisy.shape[0]
        M = self.L.flr_num_moment_planes(Q, C)
        gp, _ = self.buf(guides)
        yp, _ = self.buf(noisy)
        mp, mom = self.buf(shape=(M, H, W))
        self.check(self.L.flr_moments(ctypes.byref(p), gp, yp, mp, None), "flr_moments")
        return mom.copy()

    def solve(self, planes, p: FlrParams):
        Q, C = p.num_guides, p.num_channels
        mp, _ = self.buf(planes)
        cp, co = self.buf(shape=((Q + 1) * C,) + planes.shape[1:])
        self.check(self.L.flr_solve(ctypes.byref(p), mp, cp, None), "flr_solve")
        return co.copy()

    def apply(self, guides, coeffs, p: FlrParams):
        gp, _ = self.buf(guides)
        cp, _ = self.buf(coeffs)
        op, out = self.buf(shape=(p.num_channels,) + guides.shape[1:])
        self.check(self.L.flr_apply(ctypes.byref(p), gp, cp, op, None), "flr_apply")
        return out.copy()


def params(H, W, Q, C, r, eps=1e-3, mode=0, eps_mul=0.0, average=1, fused=1, raw=False,
           tile_rows=0):
    return FlrParams(height=H, width=W, num_guides=Q, num_channels=C, radius=r, eps=eps,
                     eps_mul=eps_mul, reg_mode=mode, average_coeffs=average, fused=fused,
                     flags=1 if raw else 0, tile_rows=tile_rows)


def _rel_err(got, want) -> float:
    """max |got - want| / max(|want|, 1e-3 rms(want))."""
    scale = max(float(np.sqrt(np.mean(np.asarray(want, np.float64) ** 2))), 1e-30)
    den = np.maximum(np.abs(want), 1e-3 * scale)
    return float(np.max(np.abs(got - want) / den))


def net_grad_errors(got, want64: dict, weights: dict) -> dict:
    """Per layer, max |got - want| over the layer's weights (and its biases)
    relative to the largest |want| of the same; got is the flat FP32 gradient
    vector in parameter order, want64 the oracle's {layer: (dW, db)}."""
    from synth.net_weights import LAYERS
    out, o = {}, 0
    for name, _, _, _ in LAYERS:
        w, b = weights[name]
        for tag, ref in (("w", want64[name][0]), ("b", want64[name][1])):
            n = ref.size
            g = np.asarray(got[o:o + n], np.float64).reshape(ref.shape)
            out[f"{name}.{tag}"] = float(np.max(np.abs(g - ref)) / max(np.max(np.abs(ref)), 1e-30))
            o += n
    assert o == len(got)
    return out


def run_case(spec: dict) -> dict:
    """Execute one case described by ``spec`` and return error figures."""
    from oracle import flr_ref as ref
    from synth import make_config, random_frame, small_integer_frame

    kind = spec["kind"]
    H, W, Q, C, r = spec["H"], spec["W"], spec["Q"], spec["C"], spec["r"]
    emu = Emu()
    try:
        if kind == "abi_checks":
            # the host dispatcher's argument checks on invalid calls (no launch)
            L = emu.L
            vp = ctypes.c_void_p
            P = ctypes.POINTER(FlrParams)
            L.flr_validate_params.argtypes = [P]
            L.flr_validate_params.restype = ctypes.c_int
            codes = []
            for field, value in [("height", 0), ("width", 40000), ("radius", -1),
                                 ("radius", 99), ("eps", float("nan")), ("eps", -1.0),
                                 ("num_guides", 0), ("num_guides", 99), ("num_channels", 9),
                                 ("reg_mode", 7), ("fused", 5), ("average_coeffs", 3),
                                 ("tile_rows", -2)]:
                p = params(8, 8, 2, 1, 2)
                setattr(p, field, value)
                codes.append(int(L.flr_validate_params(ctypes.byref(p))))
            p = params(8, 8, 2, 1, 2, fused=2)
            gp, _ = emu.buf(shape=(2, 8, 8))
            yp, _ = emu.buf(shape=(1, 8, 8))
            codes.append(int(L.flr_denoise(ctypes.byref(p), gp, yp, gp, None, 0, None)))
            codes.append(int(L.flr_denoise(ctypes.byref(p), None, yp, yp, None, 0, None)))
            codes.append(int(L.flr_denoise(ctypes.byref(p), gp + 4, yp, yp, None, 0, None)))
            return {"codes": codes}
        if kind == "raw_moments":
            fr = small_integer_frame(H, W, Q, C, seed=spec.get("seed", 0))
            p = params(H, W, Q, C, r, raw=True, tile_rows=spec.get("tile_rows", 0))
            got = emu.moments(fr["noisy"], fr["guides"], p)
            n, XtX, XtY = ref.window_moments(fr["noisy"], fr["guides"], r)
            want = [n] + [XtX[..., 0, 1 + q] for q in range(Q)] + \
                [XtY[..., 0, c] for c in range(C)] + \
                [XtX[..., 1 + a, 1 + b] for a in range(Q) for b in range(a, Q)] + \
                [XtY[..., 1 + q, c] for q in range(Q) for c in range(C)]
            want = np.stack(want)
            return {"exact": bool(np.array_equal(got.astype(np.float64), want)),
                    "maxabs": float(np.max(np.abs(got - want)))}
        if kind == "net":
            from oracle import net_ref
            from synth.net_weights import flatten_net_weights, make_net_weights
            fr = make_config(1, h=H, w=W)
            wts = make_net_weights(spec.get("seed", 2))
            got = emu.net(fr["guides"], fr["noisy"], flatten_net_weights(wts))
            want = net_ref.net_forward(fr["guides"], fr["noisy"], wts)
            d = np.abs(got - want)
            return {"maxabs": float(d.max()), "median": float(np.median(d)),
                    "within": float(np.mean(d <= 2e-3)), "shape": list(got.shape)}
        if kind == "net_trace":
            from synth.net_weights import flatten_net_weights, make_net_weights
            from tests.net_check import check_network
            fr = make_config(1, h=H, w=W)
            wts = make_net_weights(spec.get("seed", 2))
            out, acts = emu.net_trace(fr["guides"], fr["noisy"], flatten_net_weights(wts))
            plain = emu.net(fr["guides"], fr["noisy"], flatten_net_weights(wts))
            report, _ = check_network(acts, out, fr["guides"], fr["noisy"], wts)
            return {"report": report, "trace_equals_forward": bool(np.array_equal(out, plain))}
        if kind == "net_bwd_digest":
            # digest of the raw FP32 parameter gradients (to compare builds)
            import hashlib
            from synth.net_weights import flatten_net_weights, make_net_weights
            fr = make_config(1, h=H, w=W)
            wts = make_net_weights(spec.get("seed", 2))
            G = np.random.default_rng(spec.get("seed", 2) + 1).standard_normal((4, H, W))
            got = emu.net_backward(fr["guides"], fr["noisy"], flatten_net_weights(wts),
                                   G.astype(np.float32))
            return {"sha256": hashlib.sha256(np.ascontiguousarray(got, np.float32).tobytes())
                    .hexdigest(), "finite": bool(np.all(np.isfinite(got)))}
        if kind == "net_bwd":
            from oracle import net_adjoint, net_ref
            from synth.net_weights import flatten_net_weights, make_net_weights
            fr = make_config(1, h=H, w=W)
            wts = make_net_weights(spec.get("seed", 2))
            G = np.random.default_rng(spec.get("seed", 2) + 1).standard_normal((4, H, W))
            got = emu.net_backward(fr["guides"], fr["noisy"], flatten_net_weights(wts),
                                   G.astype(np.float32))
            cache = {}
            net_ref.net_forward(fr["guides"], fr["noisy"], wts, cache=cache)
            grads = net_adjoint.net_backward(cache, G.astype(np.float32).astype(np.float64))
            return net_grad_errors(got, grads, wts)
        if kind == "batch":
            from oracle import flr_lowres
            # plain frames of uneven sizes and one joint frame (noisy input and
            # low-resolution guides at 1/up of the output grid)
            sizes = spec["sizes"]
            up = spec.get("up", 2)
            frames, refs = [], []
            for k, (h, w) in enumerate(sizes):
                fr = make_config(1, seed=10 + k, h=h, w=w)
                frames.append(dict(guides=fr["guides"], noisy=fr["noisy"],
                                   tile_rows=spec.get("tile_rows", 0)))
            jh, jw = spec["joint"]
            hi = make_config(1, seed=40, h=jh, w=jw)
            lo = make_config(1, seed=40, h=jh // up, w=jw // up)
            frames.append(dict(guides=hi["guides"], guides_low=lo["guides"], noisy=lo["noisy"]))
            p = params(1, 1, 8, 3, r, 1e-3, 0, 0.0, 1, 2)
            # the persistent launch (run twice: the queue and counters reset
            # themselves), against one launch per stage, bit for bit
            got = emu.batch(frames, p, persistent_blocks=spec.get("blocks"), runs=2)
            res = {"persistent_not_failed": not emu.batch_failed}
            per_stage = emu.batch(frames, p, persistent_blocks=0)
            res["persistent_equals_stages"] = all(np.array_equal(a_, b_)
                                                  for a_, b_ in zip(got, per_stage))
            # plain frames: the same kernels and plans as flr_denoise (two-pass)
            for k, f in enumerate(frames[:-1]):
                h, w = f["guides"].shape[1:]
                one = emu.denoise(f["noisy"], f["guides"],
                                  params(h, w, 8, 3, r, 1e-3, 0, 0.0, 1, 2,
                                         tile_rows=spec.get("tile_rows", 0)))
                res[f"plain{k}_equal"] = bool(np.array_equal(got[k], one))
            # joint frame: low-resolution fit, window-averaged, bilinearly upsampled
            _, A = ref.flr_reference(lo["noisy"].astype(np.float32),
                                     lo["guides"].astype(np.float32), r,
                                     float(np.float32(1e-3)), return_coeffs=True)
            Abar = ref.average_coefficients(A, r)
            want = ref.apply_model(flr_lowres.bilinear_upsample(Abar, jh, jw, up),
                                   hi["guides"].astype(np.float32))
            res["joint_rel"] = _rel_err(got[-1], want)
            return res
        if kind == "lowres":
            from oracle import flr_lowres
            if spec.get("frame") == "config":
                fr = make_config(spec["config"], h=H, w=W)
            else:
                fr = random_frame(H, W, Q, C, seed=spec.get("seed", 0), smooth=1.5,
                                  offset=spec.get("offset", 0.0))
            noisy = fr["noisy"].astype(np.float32)
            guides = fr["guides"].astype(np.float32)
            mname = spec.get("mode", "ridge")
            eps, em = spec.get("eps", 1e-3), spec.get("eps_mul", 0.0)
            B, sig, RL = spec.get("block", 8), spec.get("sigma", 1.25), spec.get("radius_low", 4)
            p = params(H, W, Q, C, 0, eps, {"ridge": 0, "paper": 1}[mname], em, 0, 0)
            got = emu.lowres(noisy, guides, p, B, sig, RL)
            f32 = lambda v: float(np.float32(v))  # noqa: E731  (the ABI's FP32 scalars)
            want = flr_lowres.lowres_reference(noisy, guides, B, f32(sig), RL, f32(eps), mname,
                                               f32(em))
            return {"rel": _rel_err(got, want)}
        if kind == "adjoint":
            from oracle import flr_adjoint
            if spec.get("frame") == "config":
                fr = make_config(spec["config"], h=H, w=W)
            else:
                fr = random_frame(H, W, Q, C, seed=spec.get("seed", 0), smooth=1.5,
                                  offset=spec.get("offset", 0.0))
            noisy = fr["noisy"].astype(np.float32)
            guides = fr["guides"].astype(np.float32)
            G = np.random.default_rng(spec.get("seed", 0) + 11).standard_normal(
                noisy.shape).astype(np.float32)
            mname = spec.get("mode", "ridge")
            eps, em = spec.get("eps", 1e-3), spec.get("eps_mul", 0.0)
            avg = spec.get("average", 1)
            p = params(H, W, Q, C, r, eps, {"ridge": 0, "paper": 1}[mname], em, avg, 0)
            dy, dg, reg = emu.backward(noisy, guides, G, p)
            # the ABI carries eps and eps_mul as FP32: the oracle takes the same values
            ry, rg, re, rm = flr_adjoint.flr_backward(noisy, guides, G, r, float(np.float32(eps)),
                                                      mname, float(np.float32(em)), bool(avg))
            if spec.get("absolute"):
                return {"dy_max": float(np.max(np.abs(dy - ry))),
                        "dg_max": float(np.max(np.abs(dg - rg))),
                        "reg_max": float(np.max(np.abs(reg - [re, rm]))),
                        "g_max": float(np.max(np.abs(G)))}
            return {"dy_rel": _rel_err(dy, ry), "dg_rel": _rel_err(dg, rg),
                    "deps_rel": abs(reg[0] - re) / max(abs(re), 1e-30),
                    "deps_mul_abs": abs(reg[1] - rm) / max(abs(rm), 1.0)}
        if spec.get("frame") == "config":
            fr = make_config(spec["config"], h=H, w=W)
        else:
            fr = random_frame(H, W, Q, C, seed=spec.get("seed", 0), smooth=spec.get("smooth", 1.5),
                              offset=spec.get("offset", 0.0))
        noisy, guides = fr["noisy"], fr["guides"]
        mode = {"ridge": 0, "paper": 1}[spec.get("mode", "ridge")]
        eps, em = spec.get("eps", 1e-3), spec.get("eps_mul", 0.0)
        avg = spec.get("average", 1)
        tr = spec.get("tile_rows", 0)
        mname = spec.get("mode", "ridge")
        want = ref.flr_reference(noisy, guides, r, eps, mname, eps_mul=em, average=bool(avg))
        scale = max(float(np.sqrt(np.mean(want ** 2))), 1e-30)
        res = {}
        if kind in ("fused", "both"):
            got = emu.denoise(noisy, guides, params(H, W, Q, C, r, eps, mode, em, avg, 1,
                                                    tile_rows=tr))
            den = np.maximum(np.abs(want), 1e-3 * scale)
            res["fused_rel"] = float(np.max(np.abs(got - want) / den))
        if kind in ("two_pass", "both"):
            got = emu.denoise(noisy, guides, params(H, W, Q, C, r, eps, mode, em, avg, 2,
                                                    tile_rows=tr))
            den = np.maximum(np.abs(want), 1e-3 * scale)
            res["two_pass_rel"] = float(np.max(np.abs(got - want) / den))
        if kind in ("unfused", "both"):
            got = emu.denoise(noisy, guides, params(H, W, Q, C, r, eps, mode, em, avg, 0,
                                                    tile_rows=tr))
            den = np.maximum(np.abs(want), 1e-3 * scale)
            res["unfused_rel"] = float(np.max(np.abs(got - want) / den))
        if kind == "stages":
            p = params(H, W, Q, C, r, eps, mode, em, avg, 0, tile_rows=tr)
            mom = emu.moments(noisy, guides, p)
            mref = ref.central_moment_planes(noisy, guides, r)
            res["moments_err"] = float(np.max(np.abs(mom - mref)) / np.max(np.abs(mref)))
            coef = emu.solve(mref.astype(np.float32), p)
            n, Mn, Bn = ref.moments_from_central_planes(mref.astype(np.float32), Q, C)
            cref = ref.coefficient_planes(ref.solve_normalised(Mn, Bn, eps, mname, em))
            res["solve_err"] = float(np.max(np.abs(coef - cref)) / np.max(np.abs(cref)))
            out = emu.apply(guides, cref.astype(np.float32), p)
            A = ref.coefficients_from_planes(cref.astype(np.float32), Q, C)
            A = ref.average_coefficients(A, r) if avg else A
            oref = ref.apply_model(A, guides)
            res["apply_err"] = float(np.max(np.abs(out - oref)) / np.max(np.abs(oref)))
        return res
    finally:
        emu.close()


def run_in_subprocess(spec: dict, timeout: float = 600.0, sanitize: bool = False) -> dict:
    env = None
    if sanitize:
        env = sanitizer_env()
        subprocess.run([sys.executable, "-c", "from tests.cpu_emu import harness; "
                        "harness.build()"], check=True, cwd=ROOT, env=dict(env, LD_PRELOAD=""))
    res = subprocess.run([sys.executable, os.path.abspath(__file__), json.dumps(spec)],
                         stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True,
                         timeout=timeout, cwd=ROOT, env=env)
    if res.returncode != 0:
        raise RuntimeError(f"emulated case {spec} failed (rc={res.returncode}):\n"
                           f"{res.stdout[-2000:]}\n{res.stderr[-4000:]}")
    return json.loads(res.stdout.strip().splitlines()[-1])


if __name__ == "__main__":
    print(json.dumps(run_case(json.loads(sys.argv[1]))))
