"""GPU tests of batched serving (flr_batch_plan / flr_batch_run).

* Plain frames of uneven size run in one launch per stage and must equal
  flr_denoise's two-pass path frame by frame, bit for bit (the same kernels
  on the same tiles).
* A joint frame (noisy input and guides on a grid `up` times coarser) is
  compared with the oracle: the FP64 fit on the coarse grid (FP32 eps as
  the ABI carries it), window-averaged, bilinearly upsampled and applied to
  the fine guides; FP64 on the GPU too, so within 1e-6. At full size the
  oracle runs on crops: an output pixel depends on the coarse models next to
  it, and those on coarse inputs within 2r, so a 2r + 2 coarse margin is
  exact.
* The run is captured in a graph and replayed, each replay checked.
* The run is one persistent launch over a work queue; it must equal one
  launch per stage bit for bit, with the default grid and with a few
  workgroups (items then wait on items other workgroups took), and report
  no failed wait.
* The autotuner's schedule changes tiles, not results.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2410_11625_amd as flr  # noqa: E402
from oracle import flr_lowres, flr_ref  # noqa: E402
from synth import make_config  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(_dev())


def _rel(got, want):
    rms = max(float(np.sqrt(np.mean(want ** 2))), 1e-30)
    return float(np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-3 * rms)))


def _plain(h, w, seed):
    fr = make_config(1, seed=seed, h=h, w=w)
    return dict(guides=_t(fr["guides"]), noisy=_t(fr["noisy"]))


def _joint(h, w, up, seed):
    hi = make_config(1, seed=seed, h=h, w=w)
    lo = make_config(1, seed=seed, h=h // up, w=w // up)
    return (dict(guides=_t(hi["guides"]), guides_low=_t(lo["guides"]), noisy=_t(lo["noisy"])),
            hi, lo)


def _joint_oracle(hi, lo, up, r=8, crop=None):
    """Oracle output of a joint frame, or of its window crop=(y0, y1, x0, x1)
    (fine grid, multiples of up)."""
    eps = float(np.float32(1e-3))
    gl = lo["guides"].astype(np.float32)
    yl = lo["noisy"].astype(np.float32)
    gh = hi["guides"].astype(np.float32)
    if crop is None:
        y0, y1, x0, x1 = 0, gh.shape[1], 0, gh.shape[2]
    else:
        y0, y1, x0, x1 = crop
    m = 2 * r + 2
    Hl, Wl = gl.shape[1:]
    cy0, cx0 = max(y0 // up - m, 0), max(x0 // up - m, 0)
    cy1, cx1 = min(y1 // up + m, Hl), min(x1 // up + m, Wl)
    _, A = flr_ref.flr_reference(yl[:, cy0:cy1, cx0:cx1], gl[:, cy0:cy1, cx0:cx1], r, eps,
                                 return_coeffs=True)
    Abar = flr_ref.average_coefficients(A, r)
    up_A = flr_lowres.bilinear_upsample(Abar, up * (cy1 - cy0), up * (cx1 - cx0), up)
    out = flr_ref.apply_model(up_A, gh[:, up * cy0:up * cy1, up * cx0:up * cx1])
    return out[:, y0 - up * cy0:y1 - up * cy0, x0 - up * cx0:x1 - up * cx0]


def test_batch_equals_single_frames_and_joint_oracle():
    plains = [_plain(70, 300, 1), _plain(130, 517, 2), _plain(33, 256, 3), _plain(1, 260, 4)]
    jf, hi, lo = _joint(96, 600, 2, 5)
    b = flr.Batch(plains + [jf])
    outs = b.run()
    torch.cuda.synchronize()
    for f, out in zip(plains, outs):
        one = flr.denoise(f["noisy"], f["guides"], fused="two_pass")
        assert torch.equal(out, one)
    assert _rel(outs[-1].cpu().numpy(), _joint_oracle(hi, lo, 2)) <= 1e-6


def test_batch_graph_replay():
    frames = [_plain(90, 400, 6), _plain(45, 270, 7), _joint(64, 520, 2, 8)[0]]
    b = flr.Batch(frames)
    eager = [o.clone() for o in b.run()]
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.run()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        b.run()
    for _ in range(3):
        for o in b.outs:
            o.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(b.outs, eager):
            assert torch.equal(o, e)


@pytest.mark.parametrize("blocks", [None, 7])
def test_persistent_equals_per_stage(blocks):
    frames = [_plain(150, 700, 11), _plain(40, 1100, 12), _plain(9, 300, 13),
              _joint(80, 600, 2, 14)[0]]
    per_stage = [o.clone() for o in flr.Batch(frames, persistent_blocks=0).run()]
    b = flr.Batch(frames, persistent_blocks=blocks)
    assert b.plan.num_items > 0 and b.plan.persistent_blocks > 0
    for _ in range(2):  # the second run starts from the queue the first reset
        for o in b.outs:
            o.fill_(float("nan"))
        outs = b.run()
        torch.cuda.synchronize()
        for o, e in zip(outs, per_stage):
            assert torch.equal(o, e)
    assert not b.failed()


def test_workload_sizes_sampled():
    """The serving workload's frame sizes (720p, 1080p, 1440p and a joint
    1080p frame from 960x540): plain frames against flr_denoise, the joint
    frame against the oracle on crops."""
    frames = [_plain(720, 1280, 400), _plain(1080, 1920, 401), _plain(1440, 2560, 402)]
    jf, hi, lo = _joint(1080, 1920, 2, 412)
    b = flr.Batch(frames + [jf])
    outs = b.run()
    for f, out in zip(frames, outs):
        assert torch.equal(out, flr.denoise(f["noisy"], f["guides"], fused="two_pass"))
    got = outs[-1].cpu().numpy()
    for crop in [(0, 32, 0, 64), (520, 552, 900, 964), (1048, 1080, 1856, 1920)]:
        y0, y1, x0, x1 = crop
        assert _rel(got[:, y0:y1, x0:x1], _joint_oracle(hi, lo, 2, crop=crop)) <= 1e-6


def test_autotuned_schedule(tmp_path, monkeypatch):
    """The tuner's schedules (walk segment length, averaging tile height,
    batch launch schedule) change tiles, not what is computed: the batch
    equals the coefficient walk and the averaging run with the same tiles,
    bit for bit; the choices are persisted in the JSON cache and reused."""
    from paper_2410_11625_amd import autotune
    monkeypatch.setenv("FLR_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setattr(autotune, "_MEM", {})
    rows, times = autotune.tune_tile_rows(200, 700, reps=2)
    assert rows in autotune.candidate_rows(200) and rows in times
    own = autotune.tune_frames([_plain(200, 700, 9), _plain(120, 300, 10)])
    frames = autotune.tune_batch_rows(own, reps=2)
    picked = [f["tile_rows"] for f in frames]
    # each frame's own length, or one candidate length for every frame
    assert picked == [f["tile_rows"] for f in own] or (
        len(set(picked)) == 1 and picked[0] in autotune.candidate_batch_rows())
    sched = autotune.tune_batch(frames, reps=2)
    assert sched["persistent_blocks"] >= 0 and len(sched["ms"]) == 2
    b = flr.Batch(frames, persistent_blocks=sched["persistent_blocks"])
    outs = b.run()
    for f, out in zip(frames, outs):
        tr, ar = f["tile_rows"], f["apply_rows"]
        co = flr.coefficients(f["guides"], f["noisy"], 8, tile_rows=tr, intercept_pair=True)
        one = flr.apply(f["guides"], co, 8, tile_rows=ar if ar else tr, intercept_pair=True)
        assert torch.equal(out, one)
    import json
    data = json.load(open(tmp_path / "tune.json"))
    key = autotune.frame_key(200, 700, 8, 3, 8)
    assert data[key]["tile_rows"] == frames[0]["tile_rows"]
    monkeypatch.setattr(autotune, "_MEM", {})  # a new process: read back from the file
    assert autotune.tune_frame(200, 700) == data[key]
