"""The seeded input generators: determinism, shapes and value ranges."""
import hashlib

import numpy as np

from synth import make_config, make_frame, small_integer_frame


def _digest(fr):
    h = hashlib.sha256()
    for k in ("noisy", "guides", "clean"):
        h.update(np.ascontiguousarray(fr[k]).tobytes())
    return h.hexdigest()


def test_same_seed_same_frame_and_different_seed_differs():
    a = make_frame(48, 64, 7, rgb=True, fireflies=True)
    b = make_frame(48, 64, 7, rgb=True, fireflies=True)
    c = make_frame(48, 64, 8, rgb=True, fireflies=True)
    assert _digest(a) == _digest(b)
    assert _digest(a) != _digest(c)


def test_config0_shapes_and_ranges():
    fr = make_config(0)
    assert fr["noisy"].shape == (1, 256, 256) and fr["noisy"].dtype == np.float32
    assert fr["guides"].shape == (4, 256, 256)
    ao, depth, nx, ny = fr["guides"]
    assert ao.min() >= 0.0 and ao.max() <= 1.0
    assert depth.min() >= 1.0 and depth.max() <= 10.0
    assert np.all(nx * nx + ny * ny <= 1.0 + 1e-6)
    assert fr["radius"] == 8 and fr["eps"] == 1e-3
    assert np.all(fr["noisy"] >= 0)


def test_config1_shapes_fireflies_and_albedo():
    fr = make_config(1, h=216, w=384)
    assert fr["noisy"].shape == (3, 216, 384)
    assert fr["guides"].shape == (8, 216, 384)
    alb = fr["guides"][:3]
    assert alb.min() >= 0.05 and alb.max() <= 0.95
    n = fr["guides"][3:6]
    assert np.allclose((n.astype(np.float64) ** 2).sum(0), 1.0, atol=1e-5)
    # the firefly tail makes some pixels far brighter than the clean image
    ratio = fr["noisy"] / np.maximum(fr["clean"], 1e-6)
    assert ratio.max() > 20.0


def test_small_integer_frame_values():
    fr = small_integer_frame(5, 6, 3, 2, seed=1)
    assert set(np.unique(fr["guides"])) <= set(range(8))
    assert set(np.unique(fr["noisy"])) <= set(range(16))
