"""Schedule autotuner for batched serving.

Three schedule knobs are measured on the GPU (HIP events, synthetic inputs
of the frame's size) instead of taken from the launch planner's cost model:

* the coefficient walk's segment length (rows per workgroup): warm-up rows,
  which every segment repeats, against filling 256 compute units in whole
  waves of workgroups (candidates: the planner's choice and ceil(H / n) for
  n = 1..16 segments);
* the averaging tile height (rows per workgroup, at most 17): the 2r halo
  rows every tile re-reads against the number of tiles (candidates: the
  walk's segment length, which is flr_denoise's choice, and 4, 8, 12, 17);
* in a batch, one segment length for every plain frame's walk (each
  frame's own choice, or a longer one: a batch fills the GPU whatever its
  frames' segment counts, so fewer warm-up rows can win; whole batch timed);
* the batch schedule: one persistent launch over a work queue of every
  stage's tiles, or one launch per stage (whole batch timed both ways).

Results are kept in memory and in a JSON file (``FLR_AUTOTUNE_CACHE``, by
default ``~/.cache/flr_autotune.json``) keyed by the device architecture
and the frame's (H, W, Q, C, r), or for a batch schedule by the
architecture and the batch's frame list; a later process reuses them
without measuring again.
"""
from __future__ import annotations

import json
import math
import os

import torch

from .api import Batch, apply, coefficients

_MEM: dict = {}


def cache_path() -> str:
    return os.environ.get("FLR_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "flr_autotune.json"))


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key: str, value) -> None:
    _MEM[key] = value
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        data = _load()
        data[key] = value
        tmp = f"{path}.tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # an unwritable cache only costs a new measurement next time


def _lookup(key: str):
    if key not in _MEM:
        data = _load()
        if key in data:
            _MEM[key] = data[key]
    return _MEM.get(key)


def arch(device=None) -> str:
    dev = device or torch.device("cuda:0")
    return str(getattr(torch.cuda.get_device_properties(dev), "gcnArchName", "unknown"))


def frame_key(H: int, W: int, Q: int, C: int, radius: int, device=None) -> str:
    return f"{arch(device)}|frame|{H}x{W}|Q{Q}|C{C}|r{radius}"


def candidate_rows(H: int) -> list[int]:
    """0 (the planner's choice) and ceil(H / n) for n = 1..16 segments."""
    rows = {0}
    for n in range(1, 17):
        rows.add(math.ceil(H / n))
    return sorted(rows)


def candidate_apply_rows() -> list[int]:
    """0 (the walk's segment length, as flr_denoise) and fixed heights."""
    return [0, 4, 8, 12, 17]


def _time(fn, reps: int) -> float:
    fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in ev) / reps


def tune_frame(H: int, W: int, Q: int = 8, C: int = 3, radius: int = 8, eps: float = 1e-3,
               reps: int = 5, device=None) -> dict:
    """{"tile_rows", "apply_rows", "walk_ms", "apply_ms", "walk_ms_default",
    "apply_ms_default"} for an H x W frame: the fastest walk segment length,
    then the fastest averaging tile height for it (cached)."""
    key = frame_key(H, W, Q, C, radius, device)
    hit = _lookup(key)
    if hit is not None:
        return hit
    dev = device or torch.device("cuda:0")
    gen = torch.Generator(device=dev).manual_seed(0)
    g = torch.rand((Q, H, W), generator=gen, device=dev)
    y = torch.rand((C, H, W), generator=gen, device=dev)
    coeffs = torch.empty(((Q + 1) * C, H, W), device=dev)
    out = torch.empty((C, H, W), device=dev)
    walk = {rows: _time(lambda: coefficients(g, y, radius, eps=eps, tile_rows=rows, out=coeffs),
                        reps) for rows in candidate_rows(H)}
    best_walk = min(walk, key=walk.get)
    # averaging tiles: 0 means the walk's rows (the batch plan's default)
    avg = {}
    for rows in candidate_apply_rows():
        tr = rows if rows > 0 else best_walk
        avg[rows] = _time(lambda: apply(g, coeffs, radius, tile_rows=tr, out=out), reps)
    best_avg = min(avg, key=avg.get)
    res = {"tile_rows": best_walk, "apply_rows": best_avg, "walk_ms": walk[best_walk],
           "apply_ms": avg[best_avg], "walk_ms_default": walk[0], "apply_ms_default": avg[0]}
    _store(key, res)
    return res


def tune_tile_rows(H: int, W: int, Q: int = 8, C: int = 3, radius: int = 8, eps: float = 1e-3,
                   reps: int = 5, device=None) -> tuple[int, dict]:
    """(fastest walk segment length, {candidate: mean ms}) for an H x W frame
    (measured each call; tune_frame caches its results)."""
    dev = device or torch.device("cuda:0")
    gen = torch.Generator(device=dev).manual_seed(0)
    g = torch.rand((Q, H, W), generator=gen, device=dev)
    y = torch.rand((C, H, W), generator=gen, device=dev)
    coeffs = torch.empty(((Q + 1) * C, H, W), device=dev)
    times = {rows: _time(lambda: coefficients(g, y, radius, eps=eps, tile_rows=rows, out=coeffs),
                         reps) for rows in candidate_rows(H)}
    return min(times, key=times.get), times


def tune_frames(frames: list, radius: int = 8, eps: float = 1e-3) -> list:
    """The frame dicts of a batch with ``tile_rows`` and ``apply_rows`` set by
    measurement, one tuning per distinct size of the coefficient walk (the
    noisy grid)."""
    out = []
    for f in frames:
        Q = f["guides"].shape[0]
        C, h, w = f["noisy"].shape
        t = tune_frame(h, w, Q, C, radius, eps, device=f["noisy"].device)
        out.append(dict(f, tile_rows=t["tile_rows"], apply_rows=t["apply_rows"]))
    return out


def candidate_batch_rows() -> list[int]:
    """0 (each frame keeps its own walk segment length) and fixed lengths."""
    return [0, 48, 64, 96, 128]


def _batch_desc(frames: list) -> str:
    return ",".join(f"{f['noisy'].shape[1]}x{f['noisy'].shape[2]}"
                    + ("j" if f.get("guides_low") is not None else "")
                    + f"/{f.get('tile_rows', 0)}/{f.get('apply_rows', 0)}" for f in frames)


def tune_batch_rows(frames: list, radius: int = 8, eps: float = 1e-3, reps: int = 5) -> list:
    """The frames with one walk segment length for every plain frame, the
    fastest of candidate_batch_rows() for the whole batch (one launch per
    stage; cached). Joint frames are left as they are."""
    Q = frames[0]["guides"].shape[0]
    C = frames[0]["noisy"].shape[0]
    dev = frames[0]["noisy"].device
    key = f"{arch(dev)}|batchrows|Q{Q}|C{C}|r{radius}|{_batch_desc(frames)}"

    def with_rows(rows):
        if rows == 0:
            return list(frames)
        return [f if f.get("guides_low") is not None else dict(f, tile_rows=rows) for f in frames]

    hit = _lookup(key)
    if hit is None:
        times = {}
        for rows in candidate_batch_rows():
            b = Batch(with_rows(rows), radius=radius, eps=eps, persistent_blocks=0)
            times[str(rows)] = _time(b.run, reps)
        best = min(times, key=times.get)
        hit = {"rows": int(best), "ms": times}
        _store(key, hit)
    return with_rows(hit["rows"])


def tune_batch(frames: list, radius: int = 8, eps: float = 1e-3, reps: int = 5) -> dict:
    """The faster batch schedule for these frames (sizes and kinds as the
    key): {"persistent_blocks": 0 (one launch per stage) or the persistent
    grid, "ms": {str(blocks): mean ms}} (cached)."""
    desc = _batch_desc(frames)
    Q = frames[0]["guides"].shape[0]
    C = frames[0]["noisy"].shape[0]
    dev = frames[0]["noisy"].device
    key = f"{arch(dev)}|batch|Q{Q}|C{C}|r{radius}|{desc}"
    hit = _lookup(key)
    if hit is not None:
        return hit
    b = Batch(frames, radius=radius, eps=eps)
    grid = b.plan.persistent_blocks
    times = {}
    for blocks in (0, grid):
        b.plan.persistent_blocks = blocks
        times[str(blocks)] = _time(b.run, reps)
    best = min(times, key=times.get)
    res = {"persistent_blocks": int(best), "ms": times}
    _store(key, res)
    return res
