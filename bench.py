#!/usr/bin/env python3
"""Benchmark of the FLR hot path on one MI355X.

Workload: one 1920x1080 RGB frame per step (8 guides + the implied constant,
window radius 8, regulariser 1e-3, coefficients window-averaged) through the
C ABI. Inputs are seeded synthetic frames resident in HBM before timing
starts; several distinct input/output buffer sets (more than the 256 MB
Infinity Cache in total) are used in rotation so that repeated steps cannot
be served from that cache.

Paths: ``two_pass`` (default; flr_coefficients then flr_apply with the intercept pair, the fastest),
``fused`` (one kernel) and ``stages`` (flr_moments, flr_solve, flr_apply).

Prints one JSON line. Besides throughput it reports the dominant kernel's
roofline figures (its algorithmic FP64 flops over its average duration from
HIP events recorded on the launch stream) and the FP64 CPU oracle timed on a
bounded sample of the same workload. ``--copy-calibration`` also runs a
plain device copy of known size, the reference for the HBM byte counters.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

H, W, Q, C, R, EPS = 1080, 1920, 8, 3, 8, 1e-3
PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector (= 256 CU x 64 lanes x 2 x 2.4 GHz)
PEAK_HBM_GBPS = 8000.0       # MI355X HBM3E
COPY_BYTES = 1 << 30         # calibration copy: 1 GiB read + 1 GiB written


def flops_terms(Q: int, C: int) -> dict:
    """Algorithmic flops per output pixel (FMA = 2) of each step, the
    hot-path scope's count: products Q(Q+1)/2 + QC; sliding box 4 per summed
    channel (M - 1 of them, M the moment planes with the count); centring
    3 per product channel; Cholesky Q^3/3; the two triangular solves 2 Q^2 C;
    the intercepts 2QC; the coefficient average 5 per coefficient plane (FC);
    the reconstruction 2QC. Halo recomputation is not counted."""
    NP = Q * (Q + 1) // 2
    NS = Q + C + NP + Q * C          # M - 1
    FC = (Q + 1) * C
    return {
        "products": NP + Q * C,
        "box": 4 * NS,
        "centre": 3 * (NP + Q * C),
        "cholesky": Q ** 3 / 3,
        "substitution": 2 * Q * Q * C,
        "intercept": 2 * Q * C,
        "average": 5 * FC,
        "reconstruct": 2 * Q * C,
    }


def algo_flops_per_px(Q: int, C: int, part: str = "all") -> float:
    t = flops_terms(Q, C)
    if part == "coefficients":
        return sum(v for k, v in t.items() if k not in ("average", "reconstruct"))
    if part == "apply":
        return t["average"] + t["reconstruct"]
    return sum(t.values())


def algo_hbm_bytes_per_px(Q: int, C: int) -> int:
    """Algorithmic HBM bytes per pixel of the whole path: the guides and the
    noisy channels read once, the output written once (FP32)."""
    return 4 * (Q + C) + 4 * C


def kernel_source_digest() -> str:
    """Digest of the sources that define the two-pass kernels and their
    launch (the counters are void once any of them changes)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2410_11625_amd", "csrc")
    for f in ("flr_device.hpp", "flr_launch.hpp", "flr_prefix.hpp", "flr_q08.hip"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(path_name: str):
    """HBM bytes per launch of the dominant kernel, from the committed
    rocprofv3 counter summary, if it was taken on the current sources."""
    f = os.path.join(ROOT, "profiles", f"flr_{path_name}_1080p_rgb_q8_counters.json")
    if not os.path.exists(f):
        return None
    try:
        d = json.load(open(f))
    except Exception:
        return None
    if d.get("kernel_source_digest") != kernel_source_digest():
        return None
    return d.get("hbm_bytes_per_launch")


CPU_CROP = 448  # side of the square crop the oracle is timed on (about 5 s per run)
CPU_RUNS = 3


def cpu_baseline_child() -> None:
    """Runs in a child process with one BLAS/OpenMP thread: the oracle on a
    CPU_CROP x CPU_CROP crop of the 1080p workload frame, CPU_RUNS times."""
    import numpy as np
    from oracle import flr_ref
    from synth import make_config
    fr = make_config(1)
    n = CPU_CROP
    y0, x0 = (H - n) // 2, (W - n) // 2
    noisy = np.ascontiguousarray(fr["noisy"][:, y0:y0 + n, x0:x0 + n])
    guides = np.ascontiguousarray(fr["guides"][:, y0:y0 + n, x0:x0 + n])
    times = []
    for _ in range(CPU_RUNS):
        t = time.perf_counter()
        flr_ref.flr_reference(noisy, guides, R, EPS)
        times.append(time.perf_counter() - t)
    print(json.dumps({"seconds": times, "pixels": n * n}))


DOMINANT_KERNEL = {"two_pass": "walk_kernel<8, 3, 3", "fused": "walk_kernel<8, 3, 2",
                   "stages": "walk_kernel<8, 3, 0"}


def summarize_counters(fetch_csv: str, write_csv: str, path_name: str) -> int:
    """HBM bytes per launch of each kernel from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of
    ``bench.py --copy-calibration``: each counter is scaled by the ratio of
    the 1 GiB calibration copy's true bytes to what the counter read for it.
    Writes the dominant kernel's figure, with the digest of the kernel
    sources it was taken on, for the benchmark line; prints a table."""
    import csv

    def per_kernel(f):
        out = {}
        for row in csv.DictReader(open(f)):
            out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]) * 1024.0)
        return out

    fetch, write = per_kernel(fetch_csv), per_kernel(write_csv)
    # the calibration copy: the largest copy dispatches (1 GiB read, 1 GiB written)
    copies = [k for k in write if "copyBuffer" in k]
    big_w = max(v for k in copies for v in write[k])
    big_f = max(v for k in copies for v in fetch[k])
    kf, kw = COPY_BYTES / big_f, COPY_BYTES / big_w
    rows = []
    for k in sorted(set(fetch) & set(write)):
        f = kf * sum(fetch[k]) / len(fetch[k])
        w = kw * sum(write[k]) / len(write[k])
        rows.append((k, len(fetch[k]), f, w))
    print(f"calibration: FETCH_SIZE x {kf:.3f}, WRITE_SIZE x {kw:.3f} "
          f"(1 GiB copy read as {big_f / 2**20:.1f} MiB fetched, {big_w / 2**20:.1f} MiB written)")
    print("| kernel | dispatches | fetched MB | written MB |")
    print("|---|---|---|---|")
    for k, n, f, w in rows:
        print(f"| `{k[:70]}` | {n} | {f / 1e6:.1f} | {w / 1e6:.1f} |")
    dom = [r for r in rows if DOMINANT_KERNEL[path_name] in r[0]]
    if not dom:
        print("dominant kernel not found", file=sys.stderr)
        return 1
    k, n, f, w = dom[0]
    out = {"kernel": k, "kernel_source_digest": kernel_source_digest(),
           "fetch_bytes_per_launch": round(f), "write_bytes_per_launch": round(w),
           "hbm_bytes_per_launch": round(f + w),
           "calibration": {"fetch_scale": round(kf, 4), "write_scale": round(kw, 4)}}
    dst = os.path.join(ROOT, "profiles", f"flr_{path_name}_1080p_rgb_q8_counters.json")
    with open(dst, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(f"wrote {dst}")
    return 0


def time_flnr(flr, torch, np, sets, nsets, dev, stream, args):
    """FLNR per frame: guide network (BF16 MFMA) then FLR (flr_denoise,
    two-pass path) over the 8 input guides and the network's 4. Events around
    each part; the 12-guide buffers hold the input guides in planes 0..7
    (resident before timing)."""
    from synth.net_weights import flatten_net_weights, make_net_weights
    packed = flr.net_pack(torch.from_numpy(flatten_net_weights(make_net_weights(2))).to(dev))
    g12s = []
    for k in range(nsets):
        g12 = torch.empty((12, H, W), dtype=torch.float32, device=dev)
        g12[:8] = sets[k][1]
        g12s.append(g12)
    p = flr.make_params(H, W, 12, C, R, eps=EPS, average=True, fused="two_pass")
    nws = torch.empty(int(flr.api.lib().flr_net_workspace_bytes(H, W)), dtype=torch.uint8,
                      device=dev)
    rws = torch.empty(flr.workspace_bytes(p), dtype=torch.uint8, device=dev)
    outs = [torch.empty((C, H, W), dtype=torch.float32, device=dev) for _ in range(nsets)]

    def step(k, evs=None):
        noisy, guides, _ = sets[k % nsets]
        out = outs[k % nsets]             # FLR's outputs stay for its parity check
        g12 = g12s[k % nsets]
        if evs is not None:
            evs[0].record(stream)
        flr.net_forward(guides, noisy, packed, out=g12[8:], workspace=nws)
        if evs is not None:
            evs[1].record(stream)
        # flr_denoise's two-pass path over 12 guides (the regression of
        # flr_flnr_denoise): its moment walk is split into two slices
        flr.denoise(noisy, g12, radius=R, eps=EPS, average=True, fused="two_pass", out=out,
                    workspace=rws)
        if evs is not None:
            evs[2].record(stream)

    for k in range(3):
        step(k)
    torch.cuda.synchronize()
    ev = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3))
          for _ in range(args.flnr_steps)]
    for k in range(args.flnr_steps):
        step(k, ev[k])
    torch.cuda.synchronize()
    per = np.array([a.elapsed_time(c) for a, b, c in ev])
    net = np.array([a.elapsed_time(b) for a, b, c in ev])
    ms = float(np.mean(per))
    # multiply-adds per full-resolution pixel, layer by layer (half-resolution
    # layers count 1/4, quarter-resolution 1/16; exact for 1920x1080)
    macs = (11 * 16 * 9 + 16 * 16 + 16 * 32 * 9 + 32 * 32 * 9 / 4 + 32 * 64 * 9 / 4
            + 64 * 64 * 9 / 16 + 96 * 32 * 9 / 4 + 32 * 32 * 9 / 4 + 48 * 16 * 9
            + 16 * 16 * 9 + 16 * 16 * 9 + 16 * 4)
    net_flop = 2 * macs * H * W
    return {"ms_per_frame": round(ms, 5), "value": round(H * W / (ms / 1e3) / 1e6, 2),
            "unit": "Mpixel/s", "net_ms": round(float(np.mean(net)), 5),
            "regression_ms": round(float(np.mean(per - net)), 5),
            "net_tflops": round(net_flop / (float(np.mean(net)) / 1e3) / 1e12, 2),
            "net_mfma_frac_bf16": round(net_flop / (float(np.mean(net)) / 1e3) / 2.5e15, 4),
            "config": "guide net 11->4 channels (16/32/64, BF16 weights and activations, FP32 "
                      "accumulation) + FLR over 12 guides, r 8, eps 1e-3, two-pass",
            "steps": args.flnr_steps}


def time_adjoint(flr, torch, np, sets, nsets, dev, stream, args):
    """FLR adjoint per frame (flr_denoise_backward): dL/d(guides), dL/d(noisy)
    and dL/d(eps) for a resident dL/d(out), on the FLR workload's frames."""
    p = flr.make_params(H, W, Q, C, R, eps=EPS, average=True)
    ws = torch.empty(flr.backward_workspace_bytes(p), dtype=torch.uint8, device=dev)
    gen = torch.Generator(device=dev).manual_seed(5)
    gout = torch.randn((C, H, W), generator=gen, device=dev, dtype=torch.float32)
    gy = torch.empty((C, H, W), dtype=torch.float32, device=dev)
    gg = torch.empty((Q, H, W), dtype=torch.float32, device=dev)
    gr = torch.empty(2, dtype=torch.float64, device=dev)

    def step(k):
        noisy, guides, _ = sets[k % nsets]
        flr.denoise_backward(noisy, guides, gout, R, EPS, workspace=ws, grad_noisy=gy,
                             grad_guides=gg, grad_reg=gr)

    for k in range(2):
        step(k)
    torch.cuda.synchronize()
    ev = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(2))
          for _ in range(args.adjoint_steps)]
    for k in range(args.adjoint_steps):
        ev[k][0].record(stream)
        step(k)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    return {"ms_per_frame": round(ms, 5), "value": round(H * W / (ms / 1e3) / 1e6, 2),
            "unit": "Mpixel/s",
            "config": "FLR adjoint (dL/dguides, dL/dnoisy, dL/deps) of the FLR workload, FP64 "
                      "moments and fields recomputed from the inputs",
            "workspace_bytes": int(ws.numel()), "steps": args.adjoint_steps}


def time_train(flr, torch, np, dev, stream, args):
    """One FLNR training step per timed step: 8 crops of 256 x 256 (the
    training workload, inputs resident in HBM), each through the network,
    FLR over 12 guides, the L1 loss, the FLR adjoint and the network
    backward, then the AdamW update of the FP32 master weights."""
    from synth import make_training_batch
    from synth.net_weights import flatten_net_weights, make_net_weights
    crops = []
    for c in make_training_batch():
        g12 = torch.zeros((12,) + c["guides"].shape[1:], dtype=torch.float32, device=dev)
        g12[:8].copy_(torch.from_numpy(c["guides"]))
        crops.append({"guides12": g12, "noisy": torch.from_numpy(c["noisy"]).to(dev),
                      "target": torch.from_numpy(c["target"]).to(dev)})
    params = torch.from_numpy(flatten_net_weights(make_net_weights(2))).to(dev)
    tr = flr.FLNRTrainer(params, lr=1e-3)
    first = tr.step(crops).sum().item()
    tr.step(crops)
    torch.cuda.synchronize()
    ev = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(2))
          for _ in range(args.train_steps)]
    for k in range(args.train_steps):
        ev[k][0].record(stream)
        losses = tr.step(crops)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    px = sum(c["noisy"].shape[1] * c["noisy"].shape[2] for c in crops)
    return {"ms_per_step": round(ms, 4), "value": round(px / (ms / 1e3) / 1e6, 2),
            "unit": "Mpixel/s", "batch": len(crops), "crop": list(crops[0]["noisy"].shape[1:]),
            "config": "FLNR training step: network, FLR over 12 guides, L1, FLR adjoint, "
                      "network backward per crop, AdamW on FP32 master weights",
            "loss_first": round(first, 6), "loss_after": round(losses.sum().item(), 6),
            "steps": args.train_steps}


def flnr_quality(flr, torch, np, dev, args):
    """What FLNR's guides buy: the guide network trained with FLNRTrainer
    (AdamW, lr 1e-3, FLR eps fixed at 1e-3) on the training workload --
    ``args.quality_steps`` steps cycling over four batches of 8 crops of
    256 x 256 (frame seeds 100..131) -- then plain FLR, FLNR with the
    untrained network and FLNR with the trained one on held-out 1080p RGB
    frames (seeds 500, 501), each against the frame's clean shading: mean
    absolute error, relative MSE (mean of (out - clean)^2 / (clean^2 +
    0.01), the paper's rMSE form) and PSNR of both clamped to [0, 1]."""
    from synth import make_config, make_training_batch
    from synth.net_weights import flatten_net_weights, make_net_weights
    batches = []
    for k in range(4):
        crops = []
        for c in make_training_batch(seed=3 + k, frame_seed0=100 + 8 * k):
            g12 = torch.zeros((12,) + c["guides"].shape[1:], dtype=torch.float32, device=dev)
            g12[:8].copy_(torch.from_numpy(c["guides"]))
            crops.append({"guides12": g12, "noisy": torch.from_numpy(c["noisy"]).to(dev),
                          "target": torch.from_numpy(c["target"]).to(dev)})
        batches.append(crops)
    params0 = torch.from_numpy(flatten_net_weights(make_net_weights(2))).to(dev)
    params = params0.clone()
    tr = flr.FLNRTrainer(params, lr=1e-3)
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.quality_steps):
        losses.append(tr.step(batches[k % 4]).sum())
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    losses = [float(x) for x in torch.stack(losses).cpu()]

    def metrics(out, clean):
        d = out - clean
        l1 = float(d.abs().mean())
        rmse = float((d * d / (clean * clean + 0.01)).mean())
        mse01 = float(((out.clamp(0, 1) - clean.clamp(0, 1)) ** 2).mean())
        return {"l1": round(l1, 6), "rmse": round(rmse, 6),
                "psnr_db": round(10 * float(np.log10(1.0 / max(mse01, 1e-20))), 3)}

    res = {"flr": [], "flnr_untrained": [], "flnr_trained": []}
    packed0, packed = flr.net_pack(params0), flr.net_pack(params)
    for seed in (500, 501):
        fr = make_config(1, seed=seed)
        y = torch.from_numpy(fr["noisy"]).to(dev)
        g = torch.from_numpy(fr["guides"]).to(dev)
        clean = torch.from_numpy(fr["clean"].astype(np.float32)).to(dev)
        res["flr"].append(metrics(flr.denoise(y, g, radius=R, eps=EPS, fused="two_pass"), clean))
        for name, pk in (("flnr_untrained", packed0), ("flnr_trained", packed)):
            g12 = torch.zeros((12, H, W), dtype=torch.float32, device=dev)
            g12[:8] = g
            out = flr.flnr_denoise(y, g12, pk, radius=R, eps=EPS, fused="two_pass")
            res[name].append(metrics(out, clean))
    mean = {k: {m: round(float(np.mean([v[m] for v in vs])), 6) for m in vs[0]}
            for k, vs in res.items()}
    return {"train_steps": args.quality_steps, "train_s": round(train_s, 2),
            "loss_first": round(losses[0], 6), "loss_last": round(losses[-1], 6),
            "heldout_frames": 2, "mean": mean, "per_frame": res,
            "config": "FLNRTrainer (AdamW lr 1e-3, batch 8 crops of 256x256, 4 batches from "
                      "frame seeds 100..131, FLR eps 1e-3 fixed) then FLR vs FLNR on held-out "
                      "1080p RGB frames (seeds 500, 501) against the clean shading"}


def time_lowres(flr, torch, np, sets, nsets, dev, stream, args):
    """The paper's fast variant on the FLR workload's frames: 8x8 block
    moments, Gaussian sigma 1.25 (taps -4..4) at the low resolution, solve,
    bilinear model interpolation. Algorithmic HBM bytes per pixel: the
    inputs read by the block sums (4 (Q + C)), the guides read and the
    output written by the reconstruction (4 Q + 4 C); the low-resolution
    planes (1/64 of the pixels) are not counted."""
    p = flr.make_params(H, W, Q, C, 0, eps=EPS, average=False)
    ws = torch.empty(flr.lowres_workspace_bytes(p, 8, 1.25, 4), dtype=torch.uint8, device=dev)
    outs = [torch.empty((C, H, W), dtype=torch.float32, device=dev) for _ in range(nsets)]

    def step(k):
        noisy, guides, _ = sets[k % nsets]
        flr.denoise_lowres(noisy, guides, 8, 1.25, 4, eps=EPS, out=outs[k % nsets], workspace=ws)

    for k in range(3):
        step(k)
    torch.cuda.synchronize()
    ev = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(2))
          for _ in range(args.lowres_steps)]
    for k in range(args.lowres_steps):
        ev[k][0].record(stream)
        step(k)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    algo = (4 * (Q + C) + 4 * Q + 4 * C) * H * W
    gbps = algo / (ms / 1e3) / 1e9
    return {"ms_per_frame": round(ms, 5), "value": round(H * W / (ms / 1e3) / 1e6, 2),
            "unit": "Mpixel/s", "algo_hbm_bytes": algo, "hbm_algo_GBps": round(gbps, 1),
            "hbm_frac": round(gbps / PEAK_HBM_GBPS, 4),
            "config": "the paper's fast variant: 8x8 block moments, Gaussian sigma 1.25 "
                      "(taps -4..4) at 240x135, FP64 solve, bilinear models; eps 1e-3, ridge",
            "paper_rtx2080ti_ms": 0.636, "steps": args.lowres_steps}


def time_batch(flr, torch, np, sets, nsets, dev, stream, args):
    """Batched serving of 16 frames: 4 at 1280x720, 6 at 1920x1080, 4 at
    2560x1440 and 2 joint 1920x1080 frames from 960x540 noisy inputs (2x
    upsampling), 8 guides + constant, r 8, eps 1e-3. Walk segment lengths,
    averaging tile heights and the batch schedule (one persistent launch or
    one launch per stage) from the autotuner; the batch captured in a HIP
    graph and replayed; the other schedules, the planner's own choices and
    the same frames one at a time (the unbatched baseline) are timed beside
    it. Frames of one size are shifted copies of one synthetic frame
    (distinct memory, same statistics)."""
    from paper_2410_11625_amd import autotune
    from synth import make_config

    def dev_frame(fr):
        return (torch.from_numpy(fr["guides"]).to(dev), torch.from_numpy(fr["noisy"]).to(dev))

    g720, y720 = dev_frame(make_config(1, seed=400, h=720, w=1280))
    g1440, y1440 = dev_frame(make_config(1, seed=402, h=1440, w=2560))
    glo, ylo = dev_frame(make_config(1, seed=412, h=540, w=960))
    frames = []
    for k in range(4):
        frames.append(dict(guides=g720.roll(k, dims=2).contiguous(),
                           noisy=y720.roll(k, dims=2).contiguous()))
    for k in range(6):
        y, g, _ = sets[k % nsets]
        frames.append(dict(guides=g.roll(k // nsets, dims=2).contiguous(),
                           noisy=y.roll(k // nsets, dims=2).contiguous()))
    for k in range(4):
        frames.append(dict(guides=g1440.roll(k, dims=2).contiguous(),
                           noisy=y1440.roll(k, dims=2).contiguous()))
    for k in range(2):
        frames.append(dict(guides=sets[k][1], guides_low=glo.roll(k, dims=2).contiguous(),
                           noisy=ylo.roll(k, dims=2).contiguous()))
    single = autotune.tune_frames(frames, radius=R, eps=EPS)
    tuned = autotune.tune_batch_rows(single, radius=R, eps=EPS)
    sched = autotune.tune_batch(tuned, radius=R, eps=EPS)

    class OneByOne:
        """The same frames one at a time: a batch of one frame each, with
        each frame's own tuned segments (the unbatched baseline)."""
        def __init__(self, fs):
            self.bs = [flr.Batch([f], radius=R, eps=EPS, persistent_blocks=0) for f in fs]

        def run(self):
            for b1 in self.bs:
                b1.run()

    def timed(fs, blocks, graph):
        b = OneByOne(fs) if blocks == "one_by_one" else \
            flr.Batch(fs, radius=R, eps=EPS, persistent_blocks=blocks)
        for _ in range(3):
            b.run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        if not graph:
            e0.record()
            for _ in range(args.batch_steps):
                b.run()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / args.batch_steps, b
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            b.run()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            b.run()
        g.replay()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.batch_steps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.batch_steps, b

    ms, b = timed(tuned, sched["persistent_blocks"], True)
    eager_ms, _ = timed(tuned, sched["persistent_blocks"], False)
    persistent_ms, pb = timed(tuned, None, True)
    per_stage_ms, _ = timed(tuned, 0, True)
    untuned_ms, _ = timed(frames, 0, True)
    one_ms, _ = timed(single, "one_by_one", True)
    pix = sum(int(f["guides"].shape[1]) * int(f["guides"].shape[2]) for f in frames)
    rows = {f"{f['noisy'].shape[1]}x{f['noisy'].shape[2]}": [f["tile_rows"], f["apply_rows"]]
            for f in tuned}
    return {"ms_per_batch": round(ms, 5), "value": round(pix / (ms / 1e3) / 1e6, 2),
            "unit": "Mpixel/s", "frames": len(frames), "output_pixels": pix,
            "us_per_mpixel": round(ms * 1e3 / (pix / 1e6), 1),
            "eager_ms_per_batch": round(eager_ms, 5),
            "schedule": "persistent" if sched["persistent_blocks"] else "per_stage",
            "persistent_ms_per_batch": round(persistent_ms, 5),
            "persistent_workgroups": int(pb.plan.persistent_blocks),
            "persistent_items": int(pb.plan.num_items),
            "per_stage_ms_per_batch": round(per_stage_ms, 5),
            "planner_schedule_ms_per_batch": round(untuned_ms, 5),
            "one_by_one_ms": round(one_ms, 5),
            "one_by_one_us_per_mpixel": round(one_ms * 1e3 / (pix / 1e6), 1),
            "tile_rows_apply_rows": rows,
            "config": "4x1280x720 + 6x1920x1080 + 4x2560x1440 + 2 joint 1920x1080 from "
                      "960x540 (2x), 8 guides + constant, r 8, eps 1e-3; graph replay of the "
                      "tuned schedule",
            "steps": args.batch_steps}


def oracle_sampled_error(got) -> float:
    """Largest relative error of a timed output of the first buffer set (the
    seed-1 frame) against the FP64 oracle on three sampled blocks (corner,
    centre, opposite corner). Part of the CPU leg."""
    import numpy as np
    from oracle import flr_ref
    from synth import make_config
    fr0 = make_config(1, seed=1)
    errs = []
    for (y0, y1, x0, x1) in [(0, 16, 0, 32), (520, 540, 940, 972), (H - 16, H, W - 32, W)]:
        want = flr_ref.flr_reference_block(fr0["noisy"], fr0["guides"], R, EPS, y0, y1, x0, x1)
        rms = np.sqrt(np.mean(want ** 2))
        errs.append(float(np.max(np.abs(got[:, y0:y1, x0:x1] - want) /
                              np.maximum(np.abs(want), 1e-3 * rms))))
    return max(errs)


def time_path(flr, torch, np, sets, nsets, dev, stream, path, steps, warmup):
    """Time one flr_denoise execution path on the FLR workload's frames: the
    whole frame (HIP events around the timed region, on the launch stream)
    and, for the two-pass path, its first kernel separately (event between
    the two launches). Returns the path's figures with its roofline: the
    dominant kernel's algorithmic flops over its average duration against
    the FP64 (= unpacked FP32) vector peak, and the whole frame's
    algorithmic HBM bytes over the frame time against the HBM peak."""
    p = flr.make_params(H, W, Q, C, R, eps=EPS, average=True, fused=path)
    ws = torch.empty(max(flr.workspace_bytes(p), 1), dtype=torch.uint8, device=dev)
    # the two-pass path's coefficient image: intercepts as hi + lo pairs
    coeffs = torch.empty((flr.num_coeff_planes(Q, C) + C, H, W), dtype=torch.float32, device=dev)

    def step(k, evs=None):
        noisy, guides, out = sets[k % nsets]
        if evs is not None:
            evs[0].record(stream)
        if path == "two_pass":
            flr.coefficients(guides, noisy, R, eps=EPS, out=coeffs, intercept_pair=True)
            if evs is not None:
                evs[1].record(stream)
            flr.apply(guides, coeffs, R, average=True, out=out, intercept_pair=True)
        else:
            flr.denoise(noisy, guides, radius=R, eps=EPS, average=True, fused=path, out=out,
                        workspace=ws)
            if evs is not None:
                evs[1].record(stream)
        if evs is not None:
            evs[2].record(stream)

    for k in range(warmup):
        step(k)
    torch.cuda.synchronize()
    ev = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(steps)]
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for k in range(steps):
        step(k, ev[k])
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    per = np.array([a.elapsed_time(c) for a, b, c in ev])
    first = np.array([a.elapsed_time(b) for a, b, c in ev])
    pix = H * W
    if path == "two_pass":
        dom_ms = float(np.mean(first))
        dom_flops = algo_flops_per_px(Q, C, "coefficients") * pix
        dom_name = "flr_coefficients (walk_kernel<8,3,W_COEFFS>)"
        second_ms = round(float(np.mean(per - first)), 5)
    else:
        dom_ms = float(np.mean(per))
        dom_flops = algo_flops_per_px(Q, C) * pix
        dom_name = {"fused": "fused walk_kernel<8,3,W_FUSED1>",
                    "stages": "three-stage path"}[path]
        second_ms = None
    achieved = dom_flops / (dom_ms / 1e3) / 1e12
    frame_bytes = algo_hbm_bytes_per_px(Q, C) * pix
    hbm_gbps = frame_bytes / (ms / 1e3) / 1e9
    return {"path": path, "ms_per_frame": round(ms, 5),
            "value": round(pix / (ms / 1e3) / 1e6, 2), "unit": "Mpixel/s",
            "ms_per_frame_p10_p50_p90": [round(float(np.percentile(per, q)), 5)
                                         for q in (10, 50, 90)],
            "second_kernel_ms": second_ms, "steps": steps,
            "roofline": {"bound": "alu", "kernel": dom_name, "achieved": round(achieved, 3),
                         "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                         "kernel_ms": round(dom_ms, 5),
                         "algo_flops_per_launch": round(dom_flops),
                         "algo_flops_per_px": round(dom_flops / pix, 1),
                         "frame_algo_hbm_bytes": frame_bytes,
                         "hbm_algo_GBps": round(hbm_gbps, 1),
                         "hbm_frac": round(hbm_gbps / PEAK_HBM_GBPS, 4)}}


def cpu_baseline():
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[k] = "1"
    res = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child"],
                         stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env,
                         timeout=600, cwd=ROOT)
    if res.returncode != 0:
        print(res.stderr[-2000:], file=sys.stderr)
        return None
    d = json.loads(res.stdout.strip().splitlines()[-1])
    med = sorted(d["seconds"])[len(d["seconds"]) // 2]
    return {"value": round(d["pixels"] / med / 1e6, 5), "unit": "Mpixel/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"FP64 NumPy oracle (window sums as shifted adds, batched solves), a "
                       f"{CPU_CROP}x{CPU_CROP} crop of the 1080p workload frame (same guides, "
                       f"radius, eps), median of {len(d['seconds'])} runs "
                       f"({', '.join(f'{t:.2f}' for t in d['seconds'])} s) in a child process "
                       f"with OMP/OPENBLAS/MKL/NUMEXPR_NUM_THREADS=1 (one thread); host has "
                       f"{os.cpu_count()} logical CPUs")}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--path", default="two_pass", choices=["two_pass", "fused", "stages"],
                    help="flr_denoise execution path to time")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other-path", action="store_true",
                    help="skip timing the other single-frame path (fused vs two-pass)")
    ap.add_argument("--no-flnr", action="store_true", help="skip the FLNR timing")
    ap.add_argument("--flnr-steps", type=int, default=20)
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint timing")
    ap.add_argument("--no-lowres", action="store_true", help="skip the fast-variant timing")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-serving timing")
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--lowres-steps", type=int, default=50)
    ap.add_argument("--adjoint-steps", type=int, default=10)
    ap.add_argument("--no-train", action="store_true", help="skip the training-step timing")
    ap.add_argument("--no-quality", action="store_true",
                    help="skip training the guide network and measuring FLNR's quality")
    ap.add_argument("--quality-steps", type=int, default=300)
    ap.add_argument("--train-steps", type=int, default=5)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter reference)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc counter CSVs (FETCH_SIZE, WRITE_SIZE) of a "
                         "--copy-calibration run into profiles/flr_<path>_1080p_rgb_q8_counters.json")
    ap.add_argument("--cpu-baseline-child", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args(argv)

    if args.cpu_baseline_child:
        cpu_baseline_child()
        return 0
    if args.summarize_counters:
        return summarize_counters(*args.summarize_counters, args.path)
    if args.gpus != 1:
        print("bench.py: measures one GPU only (a frame is not split across GPUs; "
              "independent frames would be distributed one per GPU). Run with --gpus 1.",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2410_11625_amd as flr
    from synth import make_config

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    # Input/output sets: >= 4 and > 256 MB in total.
    per_set = (Q + 2 * C) * H * W * 4
    nsets = max(4, -(-300_000_000 // per_set))
    sets = []
    for s in range(nsets):
        if s < 2:
            fr = make_config(1, seed=1 + 1000 * s)
            sets.append((torch.from_numpy(fr["noisy"]).to(dev),
                         torch.from_numpy(fr["guides"]).to(dev),
                         torch.empty((C, H, W), dtype=torch.float32, device=dev)))
        else:  # further sets: shifted copies (distinct memory, same statistics)
            base = sets[s % 2]
            sets.append((base[0].roll(s, dims=2).contiguous(), base[1].roll(s, dims=2).contiguous(),
                         torch.empty((C, H, W), dtype=torch.float32, device=dev)))
    stream = torch.cuda.current_stream(dev)
    pix = H * W
    main_path = time_path(flr, torch, np, sets, nsets, dev, stream, args.path, args.steps,
                          args.warmup)
    ms_per_step = main_path["ms_per_frame"]
    outputs = {args.path: sets[0][2].cpu().numpy()}  # the first set's timed output
    other = None
    if not args.no_other_path:
        alt = "fused" if args.path != "fused" else "two_pass"
        other = time_path(flr, torch, np, sets, nsets, dev, stream, alt,
                          max(args.steps // 4, 10), 5)
        outputs[alt] = sets[0][2].cpu().numpy()

    # FLNR (the guide network, then FLR over 12 guides) on the same frames,
    # with the network's parameters drawn as in the workload definition
    flnr = None
    if not args.no_flnr:
        flnr = time_flnr(flr, torch, np, sets, nsets, dev, stream, args)
        flnr["vs_flr_ms"] = round(flnr["ms_per_frame"] - ms_per_step, 5)

    lowres = None
    if not args.no_lowres:
        lowres = time_lowres(flr, torch, np, sets, nsets, dev, stream, args)

    batch = None
    if not args.no_batch:
        batch = time_batch(flr, torch, np, sets, nsets, dev, stream, args)

    adjoint = None
    if not args.no_adjoint:
        adjoint = time_adjoint(flr, torch, np, sets, nsets, dev, stream, args)

    train = None
    if not args.no_train:
        train = time_train(flr, torch, np, dev, stream, args)

    quality = None
    if not args.no_quality:
        quality = flnr_quality(flr, torch, np, dev, args)
        if flnr is not None:
            quality["flnr_minus_flr_ms_per_frame"] = flnr["vs_flr_ms"]

    if args.copy_calibration:
        src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    # the CPU leg: the oracle timed on a bounded sample, and the timed
    # launches' outputs checked against it on sampled blocks
    cpu = None if args.no_cpu_baseline else cpu_baseline()
    errs = {k: oracle_sampled_error(v) for k, v in outputs.items()}
    if other is not None:
        other["max_rel_err_vs_fp64_sampled"] = errs[other["path"]]
        other["roofline"]["traffic"] = load_traffic(other["path"])
    roof = dict(main_path["roofline"])
    roof["traffic"] = load_traffic(args.path)
    line = {
        "metric": "Mpixel/s at 1080p (FLR), ms/frame, % roofline, err vs FP64",
        "value": main_path["value"],
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-io/f64-sums/f64-cholesky",
        "data": "synthetic",
        "config": {"workload": "FLR 1920x1080 RGB frame, 8 guides + constant, radius 8, "
                               "eps 1e-3, ridge, window-averaged coefficients",
                   "path": {"fused": "fused (one kernel)",
                            "two_pass": "two kernels (moments+solve, average+reconstruct)",
                            "stages": "three stages (moments, solve, apply)"}[args.path],
                   "io_dtype": "f32",
                   "accumulate_dtype": "f64 window sums, centring, Cholesky factorisation and "
                                       "substitution, intercepts and average",
                   "buffer_sets": nsets,
                   "ms_per_frame_p10_p50_p90": main_path["ms_per_frame_p10_p50_p90"],
                   "second_kernel_ms": main_path["second_kernel_ms"],
                   "max_rel_err_vs_fp64_sampled": errs[args.path],
                   "parity_ok": bool(errs[args.path] <= 1e-4)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "other_path": other,
        "flnr": flnr,
        "adjoint": adjoint,
        "lowres": lowres,
        "batch": batch,
        "train": train,
        "flnr_quality": quality,
    }
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
