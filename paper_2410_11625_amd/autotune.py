"""Schedule autotuner for batched serving.

The coefficient walk's segment length (rows per workgroup) trades warm-up
rows, which every segment repeats, against the number of workgroups, which
must fill 256 compute units in whole waves. The launch planner picks a
length from a cost model; this module measures instead: for a frame size it
times the walk on the GPU (HIP events, synthetic inputs of that size) at
the planned length and at lengths that give 1 to 16 segments, and returns
the fastest. Results are cached per (H, W, Q, C, radius).
"""
from __future__ import annotations

import math

import torch

from .api import coefficients

_CACHE: dict = {}


def candidate_rows(H: int) -> list[int]:
    """0 (the planner's choice) and ceil(H / n) for n = 1..16 segments."""
    rows = {0}
    for n in range(1, 17):
        rows.add(math.ceil(H / n))
    return sorted(rows)


def tune_tile_rows(H: int, W: int, Q: int = 8, C: int = 3, radius: int = 8, eps: float = 1e-3,
                   reps: int = 5, device=None) -> tuple[int, dict]:
    """(fastest tile_rows, {tile_rows: mean ms}) for the coefficient walk of
    an H x W frame."""
    key = (H, W, Q, C, radius)
    if key in _CACHE:
        return _CACHE[key]
    dev = device or torch.device("cuda:0")
    gen = torch.Generator(device=dev).manual_seed(0)
    g = torch.rand((Q, H, W), generator=gen, device=dev)
    y = torch.rand((C, H, W), generator=gen, device=dev)
    coeffs = torch.empty(((Q + 1) * C, H, W), device=dev)
    times = {}
    for rows in candidate_rows(H):
        coefficients(g, y, radius, eps=eps, tile_rows=rows, out=coeffs)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for a, b in ev:
            a.record()
            coefficients(g, y, radius, eps=eps, tile_rows=rows, out=coeffs)
            b.record()
        torch.cuda.synchronize()
        times[rows] = sum(a.elapsed_time(b) for a, b in ev) / reps
    best = min(times, key=times.get)
    _CACHE[key] = (best, times)
    return best, times


def tune_frames(frames: list, radius: int = 8, eps: float = 1e-3) -> list:
    """The frame dicts of a batch with ``tile_rows`` set by measurement, one
    tuning per distinct size of the coefficient walk (the noisy grid)."""
    out = []
    for f in frames:
        Q = f["guides"].shape[0]
        C, h, w = f["noisy"].shape
        rows, _ = tune_tile_rows(h, w, Q, C, radius, eps, device=f["noisy"].device)
        out.append(dict(f, tile_rows=rows))
    return out
