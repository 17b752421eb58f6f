"""Seeded random parameters for the FLNR guide network.

The network itself (Sec. 3.3, in the configuration's three-level variant) is
defined twice, independently: by the FP64 oracle and by the HIP kernels.
This module only draws its parameters: He-normal weights, std sqrt(2 /
fan_in), and small uniform biases in [-0.05, 0.05], layer by layer in a fixed
order, from ``numpy.random.default_rng(seed)``. ``LAYERS`` lists the
parameter shapes the draws are made for (name, input channels, output
channels, kernel size); it holds no arithmetic of the method.
"""
from __future__ import annotations

import numpy as np

__all__ = ["LAYERS", "make_net_weights", "flatten_net_weights"]

# (name, c_in, c_out, kernel size)
LAYERS = (
    ("in3", 11, 16, 3),
    ("in1", 16, 16, 1),
    ("e1a", 16, 32, 3),
    ("e1b", 32, 32, 3),
    ("e2a", 32, 64, 3),
    ("e2b", 64, 64, 3),
    ("d1a", 96, 32, 3),
    ("d1b", 32, 32, 3),
    ("d0a", 48, 16, 3),
    ("d0b", 16, 16, 3),
    ("out3", 16, 16, 3),
    ("out1", 16, 4, 1),
)


def make_net_weights(seed: int = 2, zero_bias: bool = False) -> dict:
    """{name: (weight [c_out][c_in][k][k] float32, bias [c_out] float32)}."""
    rng = np.random.default_rng(seed)
    out = {}
    for name, cin, cout, k in LAYERS:
        std = np.sqrt(2.0 / (cin * k * k))
        w = (rng.standard_normal((cout, cin, k, k)) * std).astype(np.float32)
        b = rng.uniform(-0.05, 0.05, cout).astype(np.float32)
        out[name] = (w, np.zeros_like(b) if zero_bias else b)
    return out


def flatten_net_weights(weights: dict) -> np.ndarray:
    """All parameters as one float32 vector, layer by layer in LAYERS order,
    each layer's weight (row-major [c_out][c_in][k][k]) followed by its bias."""
    parts = []
    for name, _, _, _ in LAYERS:
        w, b = weights[name]
        parts += [w.ravel(), b.ravel()]
    return np.concatenate(parts).astype(np.float32)
