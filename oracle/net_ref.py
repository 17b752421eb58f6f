"""FP64 reference of the FLNR guide network -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU baseline may use
this module; the product path never imports it.

The network follows Sec. 3.3 (a U-Net over the guides and the noisy input
that produces extra guide channels for the regression) in the
configuration's three-level form:

  input: the 8 guides then the 3 noisy channels, each value v compressed to
      sign(v) log(1 + |v|) (depth and radiance fireflies span decades)
  level 0 (full resolution, 16 channels):
      in3  3x3 conv 11 -> 16, ReLU
      in1  1x1 conv 16 -> 16, ReLU          = e0
  encoder:
      e1a  3x3 conv 16 -> 32, ReLU
      e1b  3x3 conv 32 -> 32, stride 2, ReLU = e1   (half resolution)
      e2a  3x3 conv 32 -> 64, ReLU
      e2b  3x3 conv 64 -> 64, stride 2, ReLU = e2   (quarter resolution)
  decoder (x2 nearest upsampling, concatenated [upsampled, skip]):
      d1a  3x3 conv up(e2) ++ e1 (96) -> 32, ReLU
      d1b  3x3 conv 32 -> 32, ReLU           = d1
      d0a  3x3 conv up(d1) ++ e0 (48) -> 16, ReLU
      d0b  3x3 conv 16 -> 16, ReLU
  output:
      out3 3x3 conv 16 -> 16, ReLU
      out1 1x1 conv 16 -> 4, sigmoid         = the 4 extra guides

Convolutions are cross-correlations with zero padding k // 2; a stride-2
layer evaluates output (i, j) at input (2i, 2j), giving ceil(n / 2) outputs;
upsampling repeats each value over a 2x2 block and is cropped to the skip
connection's size. Precision (the configuration's BF16 network): weights,
biases, the input and every activation passed between layers are rounded to
BF16 (round to nearest, ties to even); all arithmetic here is FP64 and each
layer output is rounded once. The sigmoid output is returned in FP64.
"""
from __future__ import annotations

import numpy as np

__all__ = ["bf16_round", "conv2d", "upsample2", "net_forward", "NET_LAYERS"]

# name, c_in, c_out, kernel, stride, activation (the architecture above)
NET_LAYERS = (
    ("in3", 11, 16, 3, 1, "relu"),
    ("in1", 16, 16, 1, 1, "relu"),
    ("e1a", 16, 32, 3, 1, "relu"),
    ("e1b", 32, 32, 3, 2, "relu"),
    ("e2a", 32, 64, 3, 1, "relu"),
    ("e2b", 64, 64, 3, 2, "relu"),
    ("d1a", 96, 32, 3, 1, "relu"),
    ("d1b", 32, 32, 3, 1, "relu"),
    ("d0a", 48, 16, 3, 1, "relu"),
    ("d0b", 16, 16, 3, 1, "relu"),
    ("out3", 16, 16, 3, 1, "relu"),
    ("out1", 16, 4, 1, 1, "sigmoid"),
)


def bf16_round(x) -> np.ndarray:
    """Round to the nearest BF16 value (8 significant bits, FP32 exponent
    range), ties to even, returned as float64. Zero, inf and NaN pass."""
    x = np.asarray(x, dtype=np.float64)
    out = x.copy()
    fin = np.isfinite(x) & (x != 0)
    m, e = np.frexp(x[fin])                  # x = m * 2^e, 0.5 <= |m| < 1
    # normal range: keep 8 significant bits; below 2^-126 the spacing is 2^-133
    e_eff = np.maximum(e, -125)
    scaled = np.ldexp(m, 8 + e - e_eff)       # |scaled| < 2^8
    out[fin] = np.ldexp(np.rint(scaled), e_eff - 8)
    return out


def conv2d(x: np.ndarray, w: np.ndarray, b: np.ndarray, stride: int = 1) -> np.ndarray:
    """Cross-correlation of x [c_in][H][W] with w [c_out][c_in][k][k], zero
    padding k // 2, plus bias: out[o][i][j] = b[o] + sum_{c,u,v}
    w[o][c][u][v] * x[c][stride*i + u - k//2][stride*j + v - k//2]."""
    cout, cin, k, _ = w.shape
    _, H, W = x.shape
    p = k // 2
    Ho = (H + 2 * p - k) // stride + 1
    Wo = (W + 2 * p - k) // stride + 1
    xp = np.zeros((cin, H + 2 * p, W + 2 * p))
    xp[:, p:p + H, p:p + W] = x
    out = np.broadcast_to(np.asarray(b, dtype=np.float64)[:, None, None], (cout, Ho, Wo)).copy()
    for u in range(k):
        for v in range(k):
            patch = xp[:, u:u + stride * (Ho - 1) + 1:stride, v:v + stride * (Wo - 1) + 1:stride]
            out += np.einsum("oc,chw->ohw", w[:, :, u, v].astype(np.float64), patch)
    return out


def upsample2(x: np.ndarray, H: int, W: int) -> np.ndarray:
    """Nearest x2 upsampling of x [c][h][w] cropped to [c][H][W]."""
    return x[:, np.arange(H) // 2][:, :, np.arange(W) // 2]


def net_forward(guides: np.ndarray, noisy: np.ndarray, weights: dict,
                logits: bool = False, compress: bool = True, bf16: bool = True,
                cache: dict | None = None) -> np.ndarray:
    """The 4 extra guide planes [4][H][W] for guides [8][H][W] and noisy
    [3][H][W] (float64 out). ``logits`` returns the out1 pre-activation;
    ``compress=False`` skips the input compression (for tests of the layers);
    ``bf16=False`` drops every BF16 rounding (an FP64 network, for finite-
    difference checks of gradients); ``cache``, a dict, receives each
    layer's input and pre-activation under its name (for the backward)."""
    rnd = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    wq = {n: (rnd(w), rnd(b)) for n, (w, b) in weights.items()}
    x = np.concatenate([guides, noisy]).astype(np.float64)
    if compress:
        x = np.sign(x) * np.log1p(np.abs(x))
    x = rnd(x)
    assert x.shape[0] == 11
    H, W = x.shape[1:]

    def layer(name, inp):
        spec = [l for l in NET_LAYERS if l[0] == name][0]
        _, cin, cout, k, stride, act = spec
        w, b = wq[name]
        assert w.shape == (cout, cin, k, k) and inp.shape[0] == cin, name
        z = conv2d(inp, w, b, stride)
        if cache is not None:
            cache[name] = (inp, z, w)
        if act == "relu":
            return rnd(np.maximum(z, 0.0))
        return z

    a = layer("in3", x)
    e0 = layer("in1", a)
    t = layer("e1a", e0)
    e1 = layer("e1b", t)
    t = layer("e2a", e1)
    e2 = layer("e2b", t)
    t = layer("d1a", np.concatenate([upsample2(e2, *e1.shape[1:]), e1]))
    d1 = layer("d1b", t)
    t = layer("d0a", np.concatenate([upsample2(d1, H, W), e0]))
    t = layer("d0b", t)
    t = layer("out3", t)
    z = layer("out1", t)
    if logits:
        return z
    return 1.0 / (1.0 + np.exp(-z))
