"""Pins of the FP64 guide-network backward and the FLNR training-step
gradients (oracle/net_adjoint.py), CPU only.

* Central finite differences of the FP64 network (BF16 rounding off) with
  respect to sampled weights and the bias of every layer, on a 9 x 13 frame
  (odd sizes: the stride-2 layers and the cropped upsampling take their
  ragged paths).
* Central finite differences of the FLNR L1 training loss (network -> 12
  guides -> FLR -> mean |out - target|) with respect to sampled weights,
  through the FLR adjoint.
* The upsampling adjoint as an exact dot-product identity.
* Planted mistakes in the backward fail these pins.
"""
import numpy as np
import pytest

from oracle import net_adjoint as na
from oracle import net_ref
from synth import random_frame
from synth.net_weights import make_net_weights


def _weights64():
    """The seeded weights in FP64 (finite-difference steps below FP32 resolution)."""
    return {k: (np.asarray(v[0], np.float64), np.asarray(v[1], np.float64))
            for k, v in make_net_weights(2).items()}


def _setup(H=9, W=13, seed=1):
    fr = random_frame(H, W, 8, 3, seed=seed)
    w = _weights64()
    G = np.random.default_rng(seed + 7).standard_normal((4, H, W))
    return fr, w, G


def _loss(fr, w, G):
    return float(np.sum(G * net_ref.net_forward(fr["guides"], fr["noisy"], w, bf16=False)))


def _samples(w, per_layer=2, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for name, (wt, b) in w.items():
        for _ in range(per_layer):
            out.append((name, 0, tuple(int(rng.integers(0, n)) for n in wt.shape)))
        out.append((name, 1, (int(rng.integers(0, b.shape[0])),)))
    return out


def _fd_net_ok(tol=1e-6) -> bool:
    fr, w, G = _setup()
    cache = {}
    net_ref.net_forward(fr["guides"], fr["noisy"], w, bf16=False, cache=cache)
    grads = na.net_backward(cache, G)
    h = 1e-6
    for name, which, idx in _samples(w):
        wp = {k: (v[0].copy(), v[1].copy()) for k, v in w.items()}
        wm = {k: (v[0].copy(), v[1].copy()) for k, v in w.items()}
        wp[name][which][idx] += h
        wm[name][which][idx] -= h
        fd = (_loss(fr, wp, G) - _loss(fr, wm, G)) / (2 * h)
        got = grads[name][which][idx]
        scale = max(np.max(np.abs(grads[name][which])), 1e-12)
        if abs(fd - got) > tol * scale:
            return False
    return True


def test_network_gradients_match_finite_differences():
    assert _fd_net_ok()


def test_upsample_adjoint_dot_product():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((3, 5, 7))
    dup = rng.standard_normal((3, 9, 13))
    lhs = np.sum(dup * net_ref.upsample2(x, 9, 13))
    rhs = np.sum(na.upsample2_backward(dup, 5, 7) * x)
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(dup))


def test_flnr_training_gradients_match_finite_differences():
    fr = random_frame(8, 10, 8, 3, seed=4)
    w = _weights64()
    target = np.random.default_rng(5).uniform(0.0, 2.0, fr["noisy"].shape)
    r, eps = 2, 1e-2
    loss, grads, deps = na.flnr_l1_gradients(fr["guides"], fr["noisy"], target, w, r, eps,
                                             bf16=False)
    assert np.isfinite(loss) and np.isfinite(deps)
    h = 1e-6
    for name, which, idx in _samples(w, per_layer=1, seed=3):
        wp = {k: (v[0].copy(), v[1].copy()) for k, v in w.items()}
        wm = {k: (v[0].copy(), v[1].copy()) for k, v in w.items()}
        wp[name][which][idx] += h
        wm[name][which][idx] -= h
        lp = na.flnr_l1_gradients(fr["guides"], fr["noisy"], target, wp, r, eps, bf16=False)[0]
        lm = na.flnr_l1_gradients(fr["guides"], fr["noisy"], target, wm, r, eps, bf16=False)[0]
        fd = (lp - lm) / (2 * h)
        got = grads[name][which][idx]
        scale = max(np.max(np.abs(grads[name][which])), 1e-12)
        assert abs(fd - got) <= 1e-5 * scale, (name, which, idx, fd, got)


def _upsample_mean(dup, h, w, _orig=na.upsample2_backward):
    # averages the fine gradients instead of summing them
    return _orig(dup, h, w) / 4.0


def _conv_no_stride(x, w, dz, stride, _orig=na.conv2d_backward):
    # a stride slip in the data gradient: keeps only the even input positions
    dx, dw, db = _orig(x, w, dz, stride)
    if stride == 1:
        return dx, dw, db
    dx2 = np.zeros_like(dx)
    dx2[:, ::stride, ::stride] = dx[:, ::stride, ::stride] * stride
    return dx2, dw, db


def _conv_flipped_weights(x, w, dz, stride, _orig=na.conv2d_backward):
    # uses the kernel flipped in the data gradient
    return _orig(x, w[:, :, ::-1, ::-1], dz, stride)[0], _orig(x, w, dz, stride)[1], dz.sum((1, 2))


MUTATIONS = [("upsample2_backward", _upsample_mean), ("conv2d_backward", _conv_no_stride),
             ("conv2d_backward", _conv_flipped_weights)]


@pytest.mark.parametrize("name,fn", MUTATIONS, ids=[m[1].__name__ for m in MUTATIONS])
def test_planted_backward_mistake_is_caught(monkeypatch, name, fn):
    monkeypatch.setattr(na, name, fn)
    assert not _fd_net_ok()
