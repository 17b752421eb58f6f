"""FP64 oracle of the paper's fast FLR variant -- TEST INFRASTRUCTURE ONLY.

Only the tests, the package's smoke check and the benchmark's CPU-baseline
leg may use this module; the product path never imports it.

Sec. 3.2 replaces the large full-resolution blur of the moment tensors by an
8x downsampling of the moment tensor (a strided box filter: one sum per
8x8 block), a Gaussian blur with the standard deviation divided by 8 at the
low resolution, one regularised solve per block, and bilinear interpolation
of the model parameters back to full resolution, where the model is applied
(the four stages listed there). The steps, in that order:

1. outer products x x^T and x y^T per pixel, x = [1, g] (Eq. matX);
2. block sums over B x B blocks (the last block row/column is ragged when
   the size is not a multiple of B); the constant guide's entry counts the
   pixels;
3. separable Gaussian blur of every low-resolution moment plane with
   weights exp(-d^2 / (2 sigma^2)) for |d| <= R, zero outside the low-
   resolution grid (the blurred pixel count carries the border);
4. the regularised solve of each low-resolution pixel on the moments divided
   by the blurred count (covariance scale, as the full-resolution oracle);
5. bilinear interpolation of (b, a) at each full-resolution pixel, with
   half-pixel centres (low-resolution coordinate (i + 0.5) / B - 0.5) and
   clamping at the edges; out = x^T A (Sec. 3.1).

This is a weighted least-squares fit per block (Sec. 3.2's weighted
problem): block (I, J) weights pixel p by w(I - I_p) w(J - J_p), with
(I_p, J_p) the block holding p.
"""
from __future__ import annotations

import numpy as np

from oracle.flr_ref import apply_model, design_stack, solve_normalised

__all__ = ["block_sum", "gaussian_taps", "blur_lowres", "lowres_moments", "bilinear_upsample",
           "lowres_coefficients", "lowres_reference"]


def block_sum(img: np.ndarray, B: int) -> np.ndarray:
    """Sums over B x B blocks of the last two axes -> [..., ceil(H/B), ceil(W/B)]."""
    img = np.asarray(img, dtype=np.float64)
    H, W = img.shape[-2:]
    Hl, Wl = -(-H // B), -(-W // B)
    out = np.zeros(img.shape[:-2] + (Hl, Wl))
    for I in range(Hl):
        for J in range(Wl):
            out[..., I, J] = img[..., I * B:(I + 1) * B, J * B:(J + 1) * B].sum(axis=(-2, -1))
    return out


def gaussian_taps(sigma: float, R: int) -> np.ndarray:
    """w(d) = exp(-d^2 / (2 sigma^2)) for d = -R..R (sigma = 0: only d = 0)."""
    d = np.arange(-R, R + 1, dtype=np.float64)
    if sigma == 0:
        return (d == 0).astype(np.float64)
    return np.exp(-d * d / (2.0 * sigma * sigma))


def blur_lowres(img: np.ndarray, sigma: float, R: int) -> np.ndarray:
    """Separable weighted sum over the last two axes, zero outside the grid."""
    w = gaussian_taps(sigma, R)
    img = np.asarray(img, dtype=np.float64)
    Hl, Wl = img.shape[-2:]
    tmp = np.zeros_like(img)
    for d in range(-R, R + 1):                       # along columns
        j0, j1 = max(0, -d), min(Wl, Wl - d)
        if j0 < j1:
            tmp[..., :, j0:j1] += w[d + R] * img[..., :, j0 + d:j1 + d]
    out = np.zeros_like(img)
    for d in range(-R, R + 1):                       # along rows
        i0, i1 = max(0, -d), min(Hl, Hl - d)
        if i0 < i1:
            out[..., i0:i1, :] += w[d + R] * tmp[..., i0 + d:i1 + d, :]
    return out


def lowres_moments(noisy, guides, B: int, sigma: float, R: int):
    """Blurred low-resolution X^T X [Hl,Wl,F,F], X^T Y [Hl,Wl,F,C] (steps 1-3)."""
    x = design_stack(guides)
    y = np.asarray(noisy, dtype=np.float64)
    xx = np.einsum("fhw,ghw->fghw", x, x)
    xy = np.einsum("fhw,chw->fchw", x, y)
    XtX = blur_lowres(block_sum(xx, B), sigma, R)
    XtY = blur_lowres(block_sum(xy, B), sigma, R)
    return np.moveaxis(XtX, (0, 1), (2, 3)), np.moveaxis(XtY, (0, 1), (2, 3))


def lowres_coefficients(noisy, guides, B: int, sigma: float, R: int, eps: float,
                        mode: str = "ridge", eps_mul: float = 0.0) -> np.ndarray:
    """Model per low-resolution pixel [Hl,Wl,F,C] (step 4)."""
    XtX, XtY = lowres_moments(noisy, guides, B, sigma, R)
    n = XtX[..., 0, 0][..., None, None]
    return solve_normalised(XtX / n, XtY / n, eps, mode, eps_mul)


def bilinear_upsample(A: np.ndarray, H: int, W: int, B: int) -> np.ndarray:
    """A [Hl,Wl,...] sampled at full-resolution pixel centres (step 5)."""
    Hl, Wl = A.shape[:2]

    def axis(n_full, n_low):
        u = (np.arange(n_full) + 0.5) / B - 0.5
        u = np.clip(u, 0.0, n_low - 1)
        i0 = np.floor(u).astype(int)
        i1 = np.minimum(i0 + 1, n_low - 1)
        return i0, i1, u - i0

    r0, r1, tr = axis(H, Hl)
    c0, c1, tc = axis(W, Wl)
    ex = (slice(None), slice(None)) + (None,) * (A.ndim - 2)
    top = A[r0][:, c0] * (1 - tc)[None, :][ex] + A[r0][:, c1] * tc[None, :][ex]
    bot = A[r1][:, c0] * (1 - tc)[None, :][ex] + A[r1][:, c1] * tc[None, :][ex]
    return top * (1 - tr)[:, None][ex] + bot * tr[:, None][ex]


def lowres_reference(noisy, guides, B: int = 8, sigma: float = 1.25, R: int = 4,
                     eps: float = 1e-3, mode: str = "ridge", eps_mul: float = 0.0,
                     return_coeffs: bool = False):
    """Denoised [C,H,W] in float64 (and optionally the low-resolution models)."""
    A = lowres_coefficients(noisy, guides, B, sigma, R, eps, mode, eps_mul)
    H, W = np.asarray(noisy).shape[-2:]
    out = apply_model(bilinear_upsample(A, H, W, B), guides)
    return (out, A) if return_coeffs else out
