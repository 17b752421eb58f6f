"""Pins of the FP64 oracle of the paper's fast variant (oracle/flr_lowres.py).

* brute force: each low-resolution model equals a weighted ridge least-
  squares fit built row by row from the full-resolution pixels, each with
  weight w(I - I_p) w(J - J_p) (no block sums, no separable blur, no
  moment normalisation);
* sigma = 0: independent fits per block (plain least squares per block);
* linear input (eps -> 0) is reproduced exactly, constants stay constant;
* bilinear upsampling reproduces any field linear in the low-resolution
  coordinates away from the clamped border, with half-pixel centres;
* block sums keep the total and the ragged tail;
* planted mistakes fail these pins.
"""
import numpy as np
import pytest

from oracle import flr_lowres as lr
from synth import random_frame


def _rel(a, b):
    return np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300)


def _brute(noisy, guides, B, sigma, R, eps):
    """Weighted ridge fit per low-resolution pixel from explicit rows."""
    y = np.asarray(noisy, np.float64)
    g = np.asarray(guides, np.float64)
    C, H, W = y.shape
    Q = g.shape[0]
    Hl, Wl = -(-H // B), -(-W // B)
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    X = np.concatenate([np.ones((1, H, W)), g]).reshape(Q + 1, -1).T
    Y = y.reshape(C, -1).T
    Ip, Jp = (ii // B).ravel(), (jj // B).ravel()
    A = np.zeros((Hl, Wl, Q + 1, C))
    for I in range(Hl):
        for J in range(Wl):
            dI, dJ = np.abs(Ip - I), np.abs(Jp - J)
            w = np.where((dI <= R) & (dJ <= R),
                         np.exp(-(dI ** 2 + dJ ** 2) / (2 * sigma ** 2)) if sigma > 0
                         else ((dI == 0) & (dJ == 0)).astype(float), 0.0)
            sw = np.sqrt(w)[:, None]
            # ridge on the guide coefficients in covariance scale: eps * sum(w)
            reg = np.sqrt(eps * w.sum()) * np.eye(Q + 1)[1:]
            Xa = np.vstack([sw * X, reg])
            Ya = np.vstack([sw * Y, np.zeros((Q, C))])
            A[I, J] = np.linalg.lstsq(Xa, Ya, rcond=None)[0]
    return A


CASES = [dict(H=12, W=13, B=4, sigma=1.0, R=1), dict(H=17, W=9, B=4, sigma=0.8, R=2),
         dict(H=16, W=16, B=8, sigma=1.25, R=4)]


def _battery_ok() -> bool:
    ok = True
    for c in CASES:
        fr = random_frame(c["H"], c["W"], 2, 2, seed=3, smooth=1.0, offset=1.0)
        A = lr.lowres_coefficients(fr["noisy"], fr["guides"], c["B"], c["sigma"], c["R"], 1e-2)
        Ab = _brute(fr["noisy"], fr["guides"], c["B"], c["sigma"], c["R"], 1e-2)
        ok &= _rel(A, Ab) < 1e-9
    ok &= _linear_reproduced()
    ok &= _bilinear_exact_on_linear_field()
    return bool(ok)


def _linear_reproduced() -> bool:
    fr = random_frame(20, 27, 3, 2, seed=4, smooth=1.5)
    g = fr["guides"].astype(np.float64)
    alpha = np.array([[0.7, -0.2], [1.3, 0.4], [-0.5, 2.0]])
    y = np.einsum("qhw,qc->chw", g, alpha) + np.array([0.3, -1.1])[:, None, None]
    out = lr.lowres_reference(y, g, 4, 1.25, 2, 1e-12)
    return bool(_rel(out, y) < 1e-7)


def _bilinear_exact_on_linear_field() -> bool:
    Hl, Wl, B = 5, 7, 4
    I, J = np.meshgrid(np.arange(Hl), np.arange(Wl), indexing="ij")
    A = (0.3 + 1.5 * I - 0.25 * J)[:, :, None, None] * np.ones((1, 1, 2, 3))
    up = lr.bilinear_upsample(A, Hl * B, Wl * B, B)
    u = (np.arange(Hl * B) + 0.5) / B - 0.5
    v = (np.arange(Wl * B) + 0.5) / B - 0.5
    want = 0.3 + 1.5 * u[:, None] - 0.25 * v[None, :]
    inner = (slice(B // 2, Hl * B - B // 2), slice(B // 2, Wl * B - B // 2))
    return bool(np.max(np.abs(up[..., 0, 0][inner] - want[inner])) < 1e-12)


@pytest.mark.parametrize("c", CASES, ids=lambda c: f"{c['H']}x{c['W']}-B{c['B']}-R{c['R']}")
def test_lowres_matches_brute_force_weighted_fit(c):
    fr = random_frame(c["H"], c["W"], 2, 2, seed=3, smooth=1.0, offset=1.0)
    A = lr.lowres_coefficients(fr["noisy"], fr["guides"], c["B"], c["sigma"], c["R"], 1e-2)
    Ab = _brute(fr["noisy"], fr["guides"], c["B"], c["sigma"], c["R"], 1e-2)
    assert _rel(A, Ab) < 1e-9


def test_zero_sigma_gives_independent_block_fits():
    fr = random_frame(12, 10, 2, 1, seed=5, smooth=1.0)
    A = lr.lowres_coefficients(fr["noisy"], fr["guides"], 4, 0.0, 0, 1e-2)
    Ab = _brute(fr["noisy"], fr["guides"], 4, 0.0, 0, 1e-2)
    assert _rel(A, Ab) < 1e-9
    # the first block alone
    Ab0 = _brute(fr["noisy"][:, :4, :4], fr["guides"][:, :4, :4], 4, 0.0, 0, 1e-2)
    assert _rel(A[0, 0], Ab0[0, 0]) < 1e-9


def test_linear_input_reproduced():
    assert _linear_reproduced()


def test_constant_stays_constant():
    fr = random_frame(19, 22, 3, 1, seed=6, smooth=1.0)
    y = np.full((1, 19, 22), 2.5)
    assert np.max(np.abs(lr.lowres_reference(y, fr["guides"], 8, 1.25, 4, 0.3) - 2.5)) < 1e-12


def test_bilinear_exact_on_linear_field():
    assert _bilinear_exact_on_linear_field()


def test_bilinear_constant_and_clamped_border():
    A = np.random.default_rng(1).standard_normal((3, 4, 1, 1))
    up = lr.bilinear_upsample(A, 24, 32, 8)
    # the first half block of rows/columns is clamped to the first model
    assert np.array_equal(up[:4, :4], np.broadcast_to(A[0, 0], (4, 4, 1, 1)))
    assert np.allclose(lr.bilinear_upsample(np.full((3, 4, 2, 2), 1.7), 24, 32, 8), 1.7)


def test_block_sum_total_and_ragged_tail():
    img = np.arange(5 * 7, dtype=np.float64).reshape(5, 7)
    s = lr.block_sum(img, 4)
    assert s.shape == (2, 2)
    assert s.sum() == img.sum()
    assert s[1, 1] == img[4, 4:].sum()


def test_unmutated_battery_passes():
    assert _battery_ok()


def _bilinear_no_half_pixel(A, H, W, B, _orig=lr.bilinear_upsample):
    # aligns corners instead of centres: samples at i / B
    Hl, Wl = A.shape[:2]
    u = np.clip(np.arange(H) / B, 0, Hl - 1)
    v = np.clip(np.arange(W) / B, 0, Wl - 1)
    i0, j0 = np.floor(u).astype(int), np.floor(v).astype(int)
    i1, j1 = np.minimum(i0 + 1, Hl - 1), np.minimum(j0 + 1, Wl - 1)
    tu, tv = (u - i0)[:, None, None, None], (v - j0)[None, :, None, None]
    return ((A[i0][:, j0] * (1 - tv) + A[i0][:, j1] * tv) * (1 - tu)
            + (A[i1][:, j0] * (1 - tv) + A[i1][:, j1] * tv) * tu)


def _blur_edge_replicate(img, sigma, R):
    # pads by repeating the border instead of zeros
    pad = [(0, 0)] * (img.ndim - 2) + [(R, R), (R, R)]
    p = np.pad(np.asarray(img, np.float64), pad, mode="edge")
    w = lr.gaussian_taps(sigma, R)
    Hl, Wl = img.shape[-2:]
    out = np.zeros(img.shape)
    for a in range(2 * R + 1):
        for b in range(2 * R + 1):
            out += w[a] * w[b] * p[..., a:a + Hl, b:b + Wl]
    return out


def _block_sum_drop_tail(img, B):
    img = np.asarray(img, np.float64)
    H, W = img.shape[-2:]
    Hl, Wl = -(-H // B), -(-W // B)
    out = np.zeros(img.shape[:-2] + (Hl, Wl))
    for I in range(H // B):
        for J in range(W // B):
            out[..., I, J] = img[..., I * B:(I + 1) * B, J * B:(J + 1) * B].sum(axis=(-2, -1))
    for I in range(Hl):
        for J in range(Wl):
            if I >= H // B or J >= W // B:
                out[..., I, J] = img[..., I * B:I * B + 1, J * B:J * B + 1].sum(axis=(-2, -1))
    return out


def _taps_sigma_squared(sigma, R):
    d = np.arange(-R, R + 1, dtype=np.float64)
    return np.exp(-d * d / (sigma * sigma)) if sigma else (d == 0).astype(float)


MUTATIONS = [("bilinear_upsample", _bilinear_no_half_pixel), ("blur_lowres", _blur_edge_replicate),
             ("block_sum", _block_sum_drop_tail), ("gaussian_taps", _taps_sigma_squared)]


@pytest.mark.parametrize("name,fn", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(monkeypatch, name, fn):
    monkeypatch.setattr(lr, name, fn)
    assert not _battery_ok()
