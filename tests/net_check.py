"""Layer-by-layer validity check of the BF16 guide network (Sec. 3.3) --
test infrastructure, shared by the GPU tests and the emulated-kernel tests.

The device computes every layer in FP32 on the matrix cores from BF16
inputs and rounds the result to BF16. Given the activations the device
actually fed a layer (its BF16 input, read from a forward trace), the
layer's exact output is the oracle's FP64 convolution z of those inputs
with the BF16 weights and bias; any FP32 accumulation of its K = c_in k^2
products and the bias differs from z by at most
    B = K * 2^-24 * (sum |w x| + |b|)
(one rounding of relative size 2^-24 per addition, whatever the order). As
ReLU and round-to-nearest BF16 are monotone, the device's BF16 output must
lie in [bf16(relu(z - B)), bf16(relu(z + B))]. Where that interval holds one
value (almost everywhere) the device must reproduce the oracle's BF16 value
exactly; only where z lies within B of a BF16 rounding boundary may it take
the neighbouring value (a "flip"). The prepared input is checked the same
way with the FP32 log1p's error bound, the sigmoid head to FP32 rounding of
the sigmoid of the bounded logit, and that head to 2e-3 relative as well.
"""
from __future__ import annotations

import numpy as np

from oracle import net_ref

U = 2.0 ** -24
# layer name -> (trace name of its output, trace name(s) of its input)
LAYER_IO = {
    "in3": ("in3", ("x0",)),
    "in1": ("in1", ("in3",)),
    "e1a": ("e1a", ("in1",)),
    "e1b": ("e1b", ("e1a",)),
    "e2a": ("e2a", ("e1b",)),
    "e2b": ("e2b", ("e2a",)),
    "d1a": ("d1a", ("e2b", "e1b")),   # [up2(e2), e1]
    "d1b": ("d1b", ("d1a",)),
    "d0a": ("d0a", ("d1b", "in1")),   # [up2(d1), e0]
    "d0b": ("d0b", ("d0a",)),
    "out3": ("out3", ("d0b",)),
}
SPEC = {l[0]: l for l in net_ref.NET_LAYERS}
# resolution divisor of each layer's output grid
OUT_FACTOR = {"in3": 1, "in1": 1, "e1a": 1, "e1b": 2, "e2a": 2, "e2b": 4, "d1a": 2, "d1b": 2,
              "d0a": 1, "d0b": 1, "out3": 1}


def decode_bf16(h: np.ndarray) -> np.ndarray:
    """BF16 bit patterns (int16/uint16) -> float64."""
    u = np.asarray(h).astype(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def _layer_input(name, acts, rows, cols):
    """The layer's input [c_in][len(rows)][len(cols)] at absolute input-grid
    indices rows, cols (zero outside the grid), from HWC BF16 trace tensors."""
    cin = SPEC[name][1]
    srcs = LAYER_IO[name][1]
    Hin, Win = acts[srcs[-1]].shape[:2]
    rin = (rows >= 0) & (rows < Hin)
    cinb = (cols >= 0) & (cols < Win)
    rr, cc = np.clip(rows, 0, Hin - 1), np.clip(cols, 0, Win - 1)
    if len(srcs) == 1:
        x = decode_bf16(acts[srcs[0]][rr][:, cc])[..., :cin]
    else:  # nearest x2 upsampling of the low-resolution part, then the skip
        low, skip = acts[srcs[0]], acts[srcs[1]]
        up = decode_bf16(low[rr // 2][:, cc // 2])
        x = np.concatenate([up, decode_bf16(skip[rr][:, cc])], axis=-1)[..., :cin]
    x = x * (rin[:, None, None] & cinb[None, :, None])
    return np.ascontiguousarray(np.moveaxis(x, -1, 0))


def layer_exact(name, acts, wq, y0, y1, x0, x1):
    """Exact pre-activation z and accumulation bound B of layer `name` on
    output rows [y0, y1) and columns [x0, x1), from the device's inputs."""
    _, cin, cout, k, s, _ = SPEC[name]
    w, b = wq[name]
    # input slab starting s rows/columns before the first tap centre, so that
    # the oracle's zero-padded convolution of the slab puts output y at
    # index y - y0 + 1 (its own padding is never read for those outputs)
    rows = np.arange(s * y0 - s, s * (y1 - 1) + s + 1)
    cols = np.arange(s * x0 - s, s * (x1 - 1) + s + 1)
    xin = _layer_input(name, acts, rows, cols)
    z = net_ref.conv2d(xin, w, b, s)[:, 1:1 + y1 - y0, 1:1 + x1 - x0]
    mag = net_ref.conv2d(np.abs(xin), np.abs(w), np.abs(b), s)[:, 1:1 + y1 - y0, 1:1 + x1 - x0]
    K = cin * k * k + 1
    return z, 1.01 * K * U * mag


def bf16_relu(z):
    return net_ref.bf16_round(np.maximum(z, 0.0))


def check_interval(got, z, B, what):
    """got must lie in [bf16(relu(z-B)), bf16(relu(z+B))]; returns (elements,
    elements whose interval holds two values, flips taken)."""
    lo, hi, mid = bf16_relu(z - B), bf16_relu(z + B), bf16_relu(z)
    ok = (got >= lo) & (got <= hi)
    if not ok.all():
        i = np.argwhere(~ok)[0]
        raise AssertionError(
            f"{what}: {int((~ok).sum())} of {ok.size} values outside the rounding interval; "
            f"first at {tuple(i)}: device {got[tuple(i)]!r}, oracle z {z[tuple(i)]!r} "
            f"(bound {B[tuple(i)]:.3e}), interval [{lo[tuple(i)]!r}, {hi[tuple(i)]!r}]")
    return got.size, int((lo != hi).sum()), int((got != mid).sum())


def check_prep(acts, guides, noisy, y0, y1, x0, x1):
    """x0: BF16 of sign(v) log(1 + |v|) from an FP32 log1p (OCML documents
    2 ulp; the band allows 4), padding channels exactly zero."""
    v = np.concatenate([guides, noisy])[:, y0:y1, x0:x1].astype(np.float32).astype(np.float64)
    z = np.sign(v) * np.log1p(np.abs(v))
    B = 8 * U * np.abs(z)
    got = np.moveaxis(decode_bf16(acts["x0"][y0:y1, x0:x1]), -1, 0)
    assert np.all(got[11:] == 0), "x0 padding channels are not zero"
    lo, hi = net_ref.bf16_round(z - B), net_ref.bf16_round(z + B)
    g = got[:11]
    ok = (g >= lo) & (g <= hi)
    assert ok.all(), f"x0: {int((~ok).sum())} values outside the rounding interval"
    return g.size, int((lo != hi).sum()), int((g != net_ref.bf16_round(z)).sum())


def check_head(out, acts, wq, y0, y1, x0, x1):
    """out1 + sigmoid (FP32 output) on the device's out3 activations: within
    FP32 evaluation error (8 units of 2^-24 relative) of the sigmoid over the
    logit interval, and within 2e-3 relative of the oracle's sigmoid."""
    z, B = _head_exact(acts, wq, y0, y1, x0, x1)
    sig = lambda t: 1.0 / (1.0 + np.exp(-t))  # noqa: E731
    got = np.asarray(out[:, y0:y1, x0:x1], np.float64)
    lo, hi = sig(z - B) * (1 - 8 * U), sig(z + B) * (1 + 8 * U)
    ok = (got >= lo) & (got <= hi)
    assert ok.all(), f"sigmoid head: {int((~ok).sum())} values outside the FP32 band"
    want = sig(z)
    rms = np.sqrt(np.mean(want ** 2))
    rel = np.abs(got - want) / np.maximum(np.abs(want), 1e-3 * rms)
    assert rel.max() <= 2e-3, rel.max()
    return float(rel.max()), want


def _head_exact(acts, wq, y0, y1, x0, x1):
    w, b = wq["out1"]
    x = np.moveaxis(decode_bf16(acts["out3"][y0:y1, x0:x1]), -1, 0)
    z = np.einsum("oc,chw->ohw", w[:, :, 0, 0], x) + b[:, None, None]
    mag = np.einsum("oc,chw->ohw", np.abs(w[:, :, 0, 0]), np.abs(x)) + np.abs(b)[:, None, None]
    return z, 1.01 * (16 + 1) * U * mag


def layer_region(name, acts, y0, y1, x0, x1):
    """Clip a full-resolution region to the layer's output grid."""
    Ho, Wo = acts[LAYER_IO[name][0]].shape[:2]
    f = OUT_FACTOR[name]
    return (min(y0 // f, Ho), min(-(-y1 // f), Ho), min(x0 // f, Wo), min(-(-x1 // f), Wo))


def check_network(acts, out, guides, noisy, weights, region=None):
    """Check every layer of one forward trace (acts: name -> HWC BF16 int16
    arrays; out: the FP32 sigmoid output [4][H][W]) on a full-resolution
    region (y0, y1, x0, x1), default the whole frame. Returns per-layer
    (elements, elements in a two-value interval, flips) and the head's
    largest relative error and oracle output on the region."""
    H, W = out.shape[1:]
    y0, y1, x0, x1 = region or (0, H, 0, W)
    wq = {n: (net_ref.bf16_round(w), net_ref.bf16_round(b)) for n, (w, b) in weights.items()}
    report = {"x0": check_prep(acts, guides, noisy, y0, y1, x0, x1)}
    for name in LAYER_IO:
        ly0, ly1, lx0, lx1 = layer_region(name, acts, y0, y1, x0, x1)
        if ly1 <= ly0 or lx1 <= lx0:
            continue
        z, B = layer_exact(name, acts, wq, ly0, ly1, lx0, lx1)
        got = np.moveaxis(decode_bf16(acts[LAYER_IO[name][0]][ly0:ly1, lx0:lx1]), -1, 0)
        report[name] = check_interval(got[:z.shape[0]], z, B, name)
    rel, head = check_head(out, acts, wq, y0, y1, x0, x1)
    report["head_rel"] = rel
    return report, head
