"""Planted mistakes in the oracle must be caught by its pins.

Each case swaps one oracle function for a plausibly wrong variant (off-by-one
window count, a dropped window tap, a penalised bias, a sign slip in the
Appendix regulariser, a dropped bias in the reconstruction, an unclipped
average) and checks that the battery of independent pins rejects it. All of
this runs on the CPU against the oracle only.
"""
import numpy as np
import pytest

from oracle import brute
from oracle import flr_ref as ref
from synth import random_frame, small_integer_frame


def _rel(a, b):
    return np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300)


def _battery() -> bool:
    """True when every pin holds for the (possibly mutated) oracle."""
    ok = True
    fr = small_integer_frame(6, 7, 2, 2, seed=3)
    n, XtX, XtY = ref.window_moments(fr["noisy"], fr["guides"], 2)
    nb, XtXb, XtYb = brute.brute_moments(fr["noisy"], fr["guides"], 2)
    ok &= np.array_equal(n, nb) and np.array_equal(XtX, XtXb) and np.array_equal(XtY, XtYb)
    fr = random_frame(7, 8, 2, 2, seed=4)
    for avg in (False, True):
        out, A = ref.flr_reference(fr["noisy"], fr["guides"], 2, 1e-2, average=avg,
                                   return_coeffs=True)
        outb, Ab = brute.ridge_brute(fr["noisy"], fr["guides"], 2, 1e-2, average=avg)
        ok &= _rel(out, outb) < 1e-9 and _rel(A, Ab) < 1e-8
    # Appendix compact form with a non-zero multiplicative term
    fr = random_frame(8, 8, 2, 1, seed=5, offset=1.5)
    eps, em = 1e-2, 0.3
    n, XtX, XtY = ref.window_moments(fr["noisy"], fr["guides"], 2)
    _, A = ref.flr_reference(fr["noisy"], fr["guides"], 2, eps, "paper", eps_mul=em,
                             average=False, return_coeffs=True)
    nn = n[..., None, None]
    M, B = XtX / nn, XtY / nn
    mu, nu = M[..., 0, 1:], B[..., 0, :]
    mumu = mu[..., :, None] * mu[..., None, :]
    Wc = M[..., 1:, 1:] - mumu
    Vc = B[..., 1:, :] - mu[..., :, None] * nu[..., None, :]
    Wh = Wc + em * (mumu + np.eye(2) * (mu * mu)[..., None, :]) + eps * np.eye(2)
    Hm = Wh + eps * np.eye(2) * np.diagonal(Wh, axis1=-2, axis2=-1)[..., None, :]
    ok &= _rel(A[..., 1:, :], np.linalg.solve(Hm, Vc)) < 1e-8
    # constant input stays constant
    y = np.full((1, 8, 8), 2.0)
    ok &= np.max(np.abs(ref.flr_reference(y, fr["guides"], 2, 0.3) - 2.0)) < 1e-10
    return bool(ok)


def test_unmutated_oracle_passes_battery():
    assert _battery()


def _count_plus_one(h, w, r, _orig=ref.window_count):
    return _orig(h, w, r) + 1.0


def _sum_drops_tap(img, r, _orig=ref.window_sum):
    img = np.asarray(img, dtype=np.float64)
    out = _orig(img, r)
    # forget the right-most column tap of every window
    h, w = img.shape[-2:]
    if r > 0 and w > r:
        out[..., :, : w - r] -= img[..., :, r:]
    return out


def _solve_penalise_bias(M, B, eps, mode="ridge", eps_mul=0.0, _orig=ref.solve_normalised):
    if mode == "ridge":
        mode = "raw"
    return _orig(M, B, eps, mode, eps_mul)


def _paper_sign_slip(M, B, eps, mode="ridge", eps_mul=0.0, _orig=ref.solve_normalised):
    if mode != "paper":
        return _orig(M, B, eps, mode, eps_mul)
    # (1 - eps') mu^T mu written as (1 + eps') mu^T mu
    M = np.array(M, dtype=np.float64)
    mu = M[..., 0, 1:]
    M[..., 1:, 1:] -= 2.0 * eps_mul * mu[..., :, None] * mu[..., None, :]
    return _orig(M, B, eps, mode, eps_mul)


def _apply_drops_bias(A, guides):
    g = np.asarray(guides, dtype=np.float64)
    return np.einsum("qhw,hwqc->chw", g, A[..., 1:, :])


def _average_unclipped(A, r):
    h, w = A.shape[:2]
    At = np.moveaxis(A, (0, 1), (2, 3))
    s = ref.window_sum(At, r) / float((2 * r + 1) ** 2)
    return np.moveaxis(s, (2, 3), (0, 1))


@pytest.mark.parametrize("name,fn", [
    ("window_count", _count_plus_one),
    ("window_sum", _sum_drops_tap),
    ("solve_normalised", _solve_penalise_bias),
    ("solve_normalised", _paper_sign_slip),
    ("apply_model", _apply_drops_bias),
    ("average_coefficients", _average_unclipped),
])
def test_planted_mistake_is_caught(monkeypatch, name, fn):
    monkeypatch.setattr(ref, name, fn)
    assert not _battery()
