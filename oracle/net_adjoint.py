"""FP64 backward of the FLNR guide network and the FLNR training-step
gradients -- TEST INFRASTRUCTURE ONLY.

Only the tests, the package's smoke check and the benchmark's CPU-baseline
leg may use this module; the product path never imports it.

Sec. 3.3 trains the network by backpropagating the loss of the FLNR output
through FLR into the network. This module gives, for the network of
oracle/net_ref.py, the gradients of a loss with respect to every layer's
weights and bias, by reversing the layers in the opposite order:

  sigmoid          dz = dy * s (1 - s)
  conv (k, stride) db = sum dz; dW[o,c,u,v] = sum dz[o,i,j] x[c, s i + u - p, s j + v - p];
                   dx[c, s i + u - p, s j + v - p] += W[o,c,u,v] dz[o,i,j]
  ReLU             dz = dy * [z > 0]
  upsampling x2    each coarse pixel collects the gradients of the fine
                   pixels that copied it
  concatenation    the gradient splits by channel

BF16 rounding of weights and activations is taken as the identity in the
backward (the straight-through reading): with ``bf16=True`` the gradients
are those of the FP64 network evaluated at the rounded weights and
activations; with ``bf16=False`` they are exact gradients of the FP64
network, which finite differences can check.
"""
from __future__ import annotations

import numpy as np

from oracle import flr_adjoint, flr_ref
from oracle.net_ref import NET_LAYERS, net_forward

__all__ = ["conv2d_backward", "upsample2_backward", "net_backward", "flnr_l1_gradients"]


def conv2d_backward(x, w, dz, stride: int):
    """(dx, dw, db) of z = conv2d(x, w, b, stride) (net_ref.conv2d) for dz."""
    cout, cin, k, _ = w.shape
    _, H, W = x.shape
    p = k // 2
    _, Ho, Wo = dz.shape
    xp = np.zeros((cin, H + 2 * p, W + 2 * p))
    xp[:, p:p + H, p:p + W] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w, dtype=np.float64)
    for u in range(k):
        for v in range(k):
            sl = (slice(None), slice(u, u + stride * (Ho - 1) + 1, stride),
                  slice(v, v + stride * (Wo - 1) + 1, stride))
            dw[:, :, u, v] = np.einsum("ohw,chw->oc", dz, xp[sl])
            dxp[sl] += np.einsum("oc,ohw->chw", w[:, :, u, v], dz)
    return dxp[:, p:p + H, p:p + W], dw, dz.sum(axis=(1, 2))


def upsample2_backward(dup, h: int, w: int):
    """Gradient on the coarse grid [c][h][w] of upsample2(x, H, W) for dup."""
    dx = np.zeros((dup.shape[0], h, w))
    for di in (0, 1):
        for dj in (0, 1):
            sub = dup[:, di::2, dj::2]
            dx[:, :sub.shape[1], :sub.shape[2]] += sub
    return dx


def net_backward(cache: dict, dout, logits_grad: bool = False) -> dict:
    """{layer: (dW, db)} for d(loss)/d(net output) = dout [4][H][W], given
    the cache of a net_forward call (its sigmoid output's gradient unless
    ``logits_grad``, then the logits')."""
    spec = {l[0]: l for l in NET_LAYERS}
    grads = {}

    def back(name, dact):
        """dact: gradient of the layer's output (after its activation)."""
        inp, z, w = cache[name]
        act = spec[name][5]
        if act == "relu":
            dz = dact * (z > 0)
        else:
            dz = dact
        dx, dw, db = conv2d_backward(inp, w, dz, spec[name][4])
        grads[name] = (dw, db)
        return dx

    if logits_grad:
        dz = np.asarray(dout, dtype=np.float64)
    else:
        s = 1.0 / (1.0 + np.exp(-cache["out1"][1]))
        dz = np.asarray(dout, dtype=np.float64) * s * (1.0 - s)
    d = back("out1", dz)
    d = back("out3", d)
    d = back("d0b", d)
    d = back("d0a", d)                       # input [up(d1), e0]
    nup = spec["d1b"][2]
    H0, W0 = cache["in1"][1].shape[1:]
    H1, W1 = cache["d1b"][1].shape[1:]
    dd1 = upsample2_backward(d[:nup], H1, W1)
    de0 = d[nup:]
    d = back("d1b", dd1)
    d = back("d1a", d)                       # input [up(e2), e1]
    nup = spec["e2b"][2]
    H2, W2 = cache["e2b"][1].shape[1:]
    de2 = upsample2_backward(d[:nup], H2, W2)
    de1 = d[nup:]
    d = back("e2b", de2)
    de1 = de1 + back("e2a", d)
    d = back("e1b", de1)
    de0 = de0 + back("e1a", d)
    d = back("in1", de0)
    back("in3", d)
    assert (H0, W0) == cache["in3"][1].shape[1:]
    return grads


def flnr_l1_gradients(guides, noisy, target, weights, radius: int, eps: float,
                      bf16: bool = True):
    """Loss, weight gradients and dL/deps of one FLNR training step: the
    network's 4 extra guides appended to the 8 guides, FLR over the 12
    (flr_reference, ridge, averaged), L = mean |out - target|."""
    cache = {}
    extra = net_forward(guides, noisy, weights, bf16=bf16, cache=cache)
    g12 = np.concatenate([np.asarray(guides, np.float64), extra])
    out = flr_ref.flr_reference(noisy, g12, radius, eps)
    r = out - np.asarray(target, np.float64)
    loss = float(np.mean(np.abs(r)))
    G = np.sign(r) / r.size
    _, dg12, deps, _ = flr_adjoint.flr_backward(noisy, g12, G, radius, eps)
    grads = net_backward(cache, dg12[8:])
    return loss, grads, deps
