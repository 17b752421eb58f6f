"""FP64 CPU oracle for Fast Local Regression (FLR).

TEST INFRASTRUCTURE ONLY. Nothing on the product path may import, call or
execute this module: only the tests, the package's smoke check and the
benchmark's CPU-baseline leg use it. It shares no code with the HIP library.

What it computes, step by step, in the paper's order (Sec. 3.1-3.2 and the
Appendix of "Fast Local Neural Regression for Low-Cost, Path Traced
Lambertian Global Illumination"):

1. The guide matrix of a window carries a leading column of ones and one
   column per guide (Sec. 3.1, Eq. matX); the target matrix holds the noisy
   channels (Eq. matY). The window T_k is the square of radius r centred on
   pixel k, clipped to the image, so it holds n_k in-image pixels.
2. The per-pixel matrices X_k^T X_k and X_k^T Y_k are the window sums of the
   per-pixel outer products x x^T and x y^T (Sec. 3.2: box-filtering the
   outer-product tensors yields exactly these matrices). Here the window sum
   is written out literally as a sum of (2r+1)^2 shifted images.
3. The regularised least-squares coefficients A_k (Eq. closed_form, with
   Tikhonov regularisation, Eq. tikhonov, or the Appendix normalisation).
   The regulariser is applied to the moments divided by n (covariance scale).
4. Optionally the coefficients are averaged over the same clipped window.
5. Reconstruction I_k = x_k A_k (Sec. 3.1).

Regulariser readings (the paper offers more than one):
* ``ridge``: Tikhonov on the guide coefficients only, bias unpenalised:
  (X^T X / n + eps * diag(0, 1, ..., 1)) A = X^T Y / n.
* ``paper``: the Appendix normalisation, taken literally (additive eps,
  multiplicative eps_mul, correlation-matrix solve, de-normalised output).
* ``raw``: Eq. tikhonov as written, bias penalised too:
  (X^T X / n + eps * I) A = X^T Y / n.

Arrays: ``noisy`` is [C,H,W], ``guides`` is [Q,H,W] (without the constant
guide), coefficients are [H,W,F,C] with F = Q+1 and row 0 the bias b.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "window_count", "window_sum", "design_stack", "window_moments",
    "solve_normalised", "solve_coefficients", "average_coefficients",
    "apply_model", "flr_reference", "flr_reference_block",
    "central_moment_planes", "moments_from_central_planes",
    "coefficient_planes", "coefficients_from_planes",
]


def window_count(h: int, w: int, r: int) -> np.ndarray:
    """n_k: number of in-image pixels of the clipped (2r+1)^2 window at k."""
    i = np.arange(h)
    j = np.arange(w)
    ni = np.minimum(i + r, h - 1) - np.maximum(i - r, 0) + 1
    nj = np.minimum(j + r, w - 1) - np.maximum(j - r, 0) + 1
    return (ni[:, None] * nj[None, :]).astype(np.float64)


def window_sum(img: np.ndarray, r: int) -> np.ndarray:
    """Sum over the clipped window of radius r, on the last two axes.

    Written as the literal definition: out[..., i, j] = sum of img[..., i', j']
    over |i'-i| <= r, |j'-j| <= r with (i', j') inside the image.
    """
    img = np.asarray(img, dtype=np.float64)
    h, w = img.shape[-2:]
    out = np.zeros_like(img)
    for dy in range(-r, r + 1):
        # destination rows i with source rows i+dy inside the image
        di0, di1 = max(0, -dy), min(h, h - dy)
        if di0 >= di1:
            continue
        for dx in range(-r, r + 1):
            dj0, dj1 = max(0, -dx), min(w, w - dx)
            if dj0 >= dj1:
                continue
            out[..., di0:di1, dj0:dj1] += img[..., di0 + dy:di1 + dy, dj0 + dx:dj1 + dx]
    return out


def design_stack(guides: np.ndarray) -> np.ndarray:
    """x = [1, g_1, ..., g_Q] per pixel, as [F,H,W] (Eq. matX: first column ones)."""
    g = np.asarray(guides, dtype=np.float64)
    ones = np.ones((1,) + g.shape[1:], dtype=np.float64)
    return np.concatenate([ones, g], axis=0)


def window_moments(noisy: np.ndarray, guides: np.ndarray, r: int):
    """Per-pixel X_k^T X_k [H,W,F,F], X_k^T Y_k [H,W,F,C] and n_k [H,W] (Sec. 3.2)."""
    x = design_stack(guides)
    y = np.asarray(noisy, dtype=np.float64)
    xx = np.einsum("fhw,ghw->fghw", x, x)          # outer products x x^T
    xy = np.einsum("fhw,chw->fchw", x, y)          # outer products x y^T
    XtX = np.moveaxis(window_sum(xx, r), (0, 1), (2, 3))
    XtY = np.moveaxis(window_sum(xy, r), (0, 1), (2, 3))
    n = window_count(x.shape[1], x.shape[2], r)
    return n, XtX, XtY


def solve_normalised(M: np.ndarray, B: np.ndarray, eps: float, mode: str = "ridge",
                     eps_mul: float = 0.0) -> np.ndarray:
    """Coefficients A [...,F,C] from the normalised moments M = X^T X / n, B = X^T Y / n.

    ``ridge`` and ``raw`` solve the Tikhonov-regularised normal equations
    (Eq. tikhonov); ``paper`` follows the Appendix steps literally.
    """
    M = np.asarray(M, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    F = M.shape[-1]
    if mode in ("ridge", "raw"):
        pen = np.eye(F)
        if mode == "ridge":
            pen[0, 0] = 0.0
        return np.linalg.solve(M + eps * pen, B)
    if mode != "paper":
        raise ValueError(f"unknown mode {mode!r}")
    # Appendix: X^T X split into n (top-left), u_X (first row/column) and S.
    # With the moments already divided by n, the top-left entry is 1 and
    # u_X / n is the window mean of each guide.
    mu = M[..., 0, 1:]                                # mu_X = u_X / n
    S_n = M[..., 1:, 1:]                              # S / n
    mumu = mu[..., :, None] * mu[..., None, :]        # mu_X^T mu_X (outer product)
    Q = F - 1
    eye = np.eye(Q)
    # W_hat = S/n + eps' diag(mu^T mu) + eps I - (1 - eps') mu^T mu
    diag_mumu = eye * (mu * mu)[..., None, :]
    W_hat = S_n + eps_mul * diag_mumu + eps * eye - (1.0 - eps_mul) * mumu
    sig = np.sqrt(np.diagonal(W_hat, axis1=-2, axis2=-1))   # sigma_hat
    C_hat = W_hat / (sig[..., :, None] * sig[..., None, :])
    mu_y = B[..., 0, :]                                # top row of X^T Y / n
    B_hat = (B[..., 1:, :] - mu[..., :, None] * mu_y[..., None, :]) / sig[..., :, None]
    A_hat = np.linalg.solve(C_hat + eps * eye, B_hat)
    # y = ((x - mu)/sigma_hat) A_hat + mu_Y  =  b + x^T a  with
    a = A_hat / sig[..., :, None]
    b = mu_y - np.einsum("...q,...qc->...c", mu, a)
    return np.concatenate([b[..., None, :], a], axis=-2)


def solve_coefficients(n, XtX, XtY, eps: float, mode: str = "ridge", eps_mul: float = 0.0):
    """A_k for every pixel from the window moments (regulariser in covariance scale)."""
    nn = np.asarray(n, dtype=np.float64)[..., None, None]
    return solve_normalised(XtX / nn, XtY / nn, eps, mode, eps_mul)


def average_coefficients(A: np.ndarray, r: int) -> np.ndarray:
    """Mean of A_k over the clipped window T_i of each pixel i."""
    h, w = A.shape[:2]
    At = np.moveaxis(A, (0, 1), (2, 3))               # [F,C,H,W]
    s = window_sum(At, r) / window_count(h, w, r)
    return np.moveaxis(s, (2, 3), (0, 1))


def apply_model(A: np.ndarray, guides: np.ndarray) -> np.ndarray:
    """I_k = x_k A_k with x_k = [1, g(k)] (Sec. 3.1); returns [C,H,W]."""
    x = design_stack(guides)
    return np.einsum("fhw,hwfc->chw", x, A)


def flr_reference(noisy, guides, radius: int, eps: float, mode: str = "ridge",
                  eps_mul: float = 0.0, average: bool = True, return_coeffs: bool = False):
    """Denoised [C,H,W] in float64 (and optionally the unaveraged coefficients)."""
    n, XtX, XtY = window_moments(noisy, guides, radius)
    A = solve_coefficients(n, XtX, XtY, eps, mode, eps_mul)
    Abar = average_coefficients(A, radius) if average else A
    out = apply_model(Abar, guides)
    return (out, A) if return_coeffs else out


def flr_reference_block(noisy, guides, radius: int, eps: float, y0: int, y1: int,
                        x0: int, x1: int, **kw):
    """Output rows [y0,y1) and columns [x0,x1) of ``flr_reference`` on the full frame.

    The output at a pixel depends only on inputs within 2r of it (r for the
    moments, r more for the coefficient average), and window clipping only
    depends on the image borders. So it is evaluated on the crop extended by
    2r (clamped to the image); pixels at least 2r from a crop edge that is not
    an image edge are identical to the full-frame result.
    """
    H, W = noisy.shape[-2:]
    m = 2 * radius
    cy0, cy1 = max(0, y0 - m), min(H, y1 + m)
    cx0, cx1 = max(0, x0 - m), min(W, x1 + m)
    out = flr_reference(noisy[:, cy0:cy1, cx0:cx1], guides[:, cy0:cy1, cx0:cx1],
                        radius, eps, **kw)
    return out[:, y0 - cy0:y1 - cy0, x0 - cx0:x1 - cx0]


# ---------------------------------------------------------------------------
# Plane layouts used by the library's stage entry points, produced here from
# the definition-level quantities above (so the stages can be checked one by
# one).

def central_moment_planes(noisy, guides, radius: int) -> np.ndarray:
    """[M,H,W]: n | mean of each guide | mean of each channel |
    guide covariance, upper triangle row-major | guide-channel covariance [q][c].

    Covariances are window second moments divided by n minus the product of
    the means (the Appendix's W = S/n - mu^T mu, and its X^T Y analogue).
    """
    n, XtX, XtY = window_moments(noisy, guides, radius)
    F = XtX.shape[-1]
    Q = F - 1
    C = XtY.shape[-1]
    nn = n[..., None, None]
    M = XtX / nn
    B = XtY / nn
    mu = M[..., 0, 1:]
    nu = B[..., 0, :]
    Wc = M[..., 1:, 1:] - mu[..., :, None] * mu[..., None, :]
    Vc = B[..., 1:, :] - mu[..., :, None] * nu[..., None, :]
    planes = [n]
    planes += [mu[..., q] for q in range(Q)]
    planes += [nu[..., c] for c in range(C)]
    planes += [Wc[..., p, q] for p in range(Q) for q in range(p, Q)]
    planes += [Vc[..., q, c] for q in range(Q) for c in range(C)]
    return np.stack(planes)


def moments_from_central_planes(planes: np.ndarray, Q: int, C: int):
    """Inverse of ``central_moment_planes``: (n, X^T X / n, X^T Y / n)."""
    planes = np.asarray(planes, dtype=np.float64)
    H, W = planes.shape[-2:]
    k = 0
    n = planes[k]; k += 1
    mu = np.moveaxis(planes[k:k + Q], 0, -1); k += Q
    nu = np.moveaxis(planes[k:k + C], 0, -1); k += C
    Wc = np.zeros((H, W, Q, Q))
    for p in range(Q):
        for q in range(p, Q):
            Wc[..., p, q] = planes[k]
            Wc[..., q, p] = planes[k]
            k += 1
    Vc = np.zeros((H, W, Q, C))
    for q in range(Q):
        for c in range(C):
            Vc[..., q, c] = planes[k]
            k += 1
    F = Q + 1
    M = np.zeros((H, W, F, F))
    M[..., 0, 0] = 1.0
    M[..., 0, 1:] = mu
    M[..., 1:, 0] = mu
    M[..., 1:, 1:] = Wc + mu[..., :, None] * mu[..., None, :]
    B = np.zeros((H, W, F, C))
    B[..., 0, :] = nu
    B[..., 1:, :] = Vc + mu[..., :, None] * nu[..., None, :]
    return n, M, B


def coefficient_planes(A: np.ndarray) -> np.ndarray:
    """[F*C,H,W]: b[c] for each channel, then a[q][c] row-major."""
    F, C = A.shape[-2:]
    return np.stack([A[..., f, c] for f in range(F) for c in range(C)])


def coefficients_from_planes(planes: np.ndarray, Q: int, C: int) -> np.ndarray:
    planes = np.asarray(planes, dtype=np.float64)
    F = Q + 1
    H, W = planes.shape[-2:]
    A = np.zeros((H, W, F, C))
    for f in range(F):
        for c in range(C):
            A[..., f, c] = planes[f * C + c]
    return A
