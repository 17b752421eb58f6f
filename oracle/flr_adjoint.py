"""FP64 adjoint (reverse-mode gradient) of the FLR oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the package's smoke check and the benchmark's CPU-baseline
leg may use this module; the product path never imports it.

FLR is differentiable end to end (Sec. 3 and Sec. 3.3: the network behind the
guides is trained through it; the Appendix learns its regularisers by
backpropagation). Given dL/d(out) for out = flr_reference(noisy, guides, r,
eps, mode, eps_mul, average), this module returns dL/d(noisy), dL/d(guides),
dL/d(eps) and dL/d(eps_mul). Each function below is the reverse of one step
of the forward oracle, taken in the reverse order and in the forward oracle's
own (uncentred) quantities:

  forward                                     reverse
  1 XtX = wsum(x x^T), XtY = wsum(x y^T)      moments_adjoint
  2 M = XtX / n, B = XtY / n                  (division by n)
  3 A = solve(M, B; eps, mode, eps_mul)       solve_vjp (Tikhonov or Appendix)
  4 Abar = wsum(A) / n   (if averaging)       averaging_adjoint
  5 out = x^T Abar                            reconstruction_adjoint

with x = [1, g] (Eq. matX) and wsum the clipped window sum. The window sum
is its own adjoint: pixel k is in the window of i exactly when i is in the
window of k. Matrix identities used: for A = K^-1 B with K symmetric,
dB = K^-1 dA and dK = -dB A^T.
"""
from __future__ import annotations

import numpy as np

from oracle.flr_ref import (average_coefficients, design_stack, solve_normalised, window_count, window_moments,
                             window_sum)

__all__ = ["reconstruction_adjoint", "averaging_adjoint", "solve_vjp", "moments_adjoint",
           "flr_backward"]


def reconstruction_adjoint(Abar: np.ndarray, x: np.ndarray, G: np.ndarray):
    """out_c = sum_f x_f Abar_fc (Sec. 3.1). Returns dAbar [H,W,F,C] and the
    direct part of dx [F,H,W]."""
    dAbar = np.einsum("fhw,chw->hwfc", x, G)
    dx = np.einsum("hwfc,chw->fhw", Abar, G)
    return dAbar, dx


def averaging_adjoint(dAbar: np.ndarray, r: int) -> np.ndarray:
    """Abar_i = (1/n_i) sum_{k in T_i} A_k  ->  dA_k = sum_{i in T_k} dAbar_i / n_i."""
    h, w = dAbar.shape[:2]
    t = np.moveaxis(dAbar, (0, 1), (2, 3)) / window_count(h, w, r)
    return np.moveaxis(window_sum(t, r), (2, 3), (0, 1))


def _tikhonov_vjp(M, B, dA, eps, pen):
    """A = (M + eps P)^-1 B (Eq. tikhonov; P = I, or I without the bias entry)."""
    K = M + eps * pen
    A = np.linalg.solve(K, B)
    dB = np.linalg.solve(K, dA)                       # K is symmetric
    dK = -np.einsum("...fc,...gc->...fg", dB, A)
    deps = float(np.sum(dK * pen))
    return dK, dB, deps, 0.0


def _paper_vjp(M, B, dA, eps, em):
    """Reverse of the Appendix steps as the forward oracle takes them:
    W^ = S/n + eps' diag(mu o mu) + eps I - (1 - eps') mu mu^T,
    sigma = sqrt(diag W^), C^ = W^ / (sigma sigma^T), B^ = (B_g - mu nu^T) / sigma,
    A^ = (C^ + eps I)^-1 B^, a = A^ / sigma, b = nu - a^T mu."""
    F = M.shape[-1]
    Q = F - 1
    eye = np.eye(Q)
    # forward quantities
    mu = M[..., 0, 1:]
    S_n = M[..., 1:, 1:]
    mumu = mu[..., :, None] * mu[..., None, :]
    diag_mumu = eye * (mu * mu)[..., None, :]
    W_hat = S_n + em * diag_mumu + eps * eye - (1.0 - em) * mumu
    sig = np.sqrt(np.diagonal(W_hat, axis1=-2, axis2=-1))
    ss = sig[..., :, None] * sig[..., None, :]
    C_hat = W_hat / ss
    mu_y = B[..., 0, :]
    Bc = B[..., 1:, :] - mu[..., :, None] * mu_y[..., None, :]
    B_hat = Bc / sig[..., :, None]
    K = C_hat + eps * eye
    A_hat = np.linalg.solve(K, B_hat)
    a = A_hat / sig[..., :, None]
    # reverse
    db = dA[..., 0, :]
    da = dA[..., 1:, :]
    dmu_y = db.copy()                                              # b = nu - a^T mu
    dmu = -np.einsum("...qc,...c->...q", a, db)
    da = da - mu[..., :, None] * db[..., None, :]
    dA_hat = da / sig[..., :, None]                                # a = A^ / sigma
    dsig = -np.sum(da * A_hat, axis=-1) / sig ** 2
    dB_hat = np.linalg.solve(K, dA_hat)                            # A^ = K^-1 B^
    dK = -np.einsum("...pc,...qc->...pq", dB_hat, A_hat)
    deps = float(np.sum(np.trace(dK, axis1=-2, axis2=-1)))        # K = C^ + eps I
    dC = dK
    dBc = dB_hat / sig[..., :, None]                               # B^ = Bc / sigma
    dsig -= np.sum(dB_hat * Bc, axis=-1) / sig ** 2
    dB = np.zeros_like(B)
    dB[..., 1:, :] = dBc                                           # Bc = B_g - mu nu^T
    dmu -= np.einsum("...qc,...c->...q", dBc, mu_y)
    dmu_y -= np.einsum("...qc,...q->...c", dBc, mu)
    dW_hat = dC / ss                                               # C^ = W^ / (s s^T)
    t = dC * C_hat
    dsig -= (np.sum(t, axis=-1) + np.sum(t, axis=-2)) / sig
    dW_hat = dW_hat + eye * (dsig / (2.0 * sig))[..., None, :]     # sigma = sqrt(diag W^)
    # W^ = S/n + eps' diag(mu o mu) + eps I - (1 - eps') mu mu^T
    deps += float(np.sum(np.trace(dW_hat, axis1=-2, axis2=-1)))
    dem = float(np.sum(dW_hat * (diag_mumu + mumu)))
    dd = np.diagonal(dW_hat, axis1=-2, axis2=-1)
    dmu += em * 2.0 * dd * mu
    dmu -= (1.0 - em) * np.einsum("...pq,...q->...p", dW_hat + np.swapaxes(dW_hat, -1, -2), mu)
    dM = np.zeros_like(M)
    dM[..., 1:, 1:] = dW_hat
    dM[..., 0, 1:] = dmu                                           # mu is read from row 0
    dB[..., 0, :] += dmu_y
    return dM, dB, deps, dem


def solve_vjp(M, B, dA, eps: float, mode: str = "ridge", eps_mul: float = 0.0):
    """dL/dM, dL/dB, dL/deps, dL/deps_mul for A = solve_normalised(M, B, ...)."""
    M = np.asarray(M, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    F = M.shape[-1]
    if mode in ("ridge", "raw"):
        pen = np.eye(F)
        if mode == "ridge":
            pen[0, 0] = 0.0
        return _tikhonov_vjp(M, B, dA, eps, pen)
    if mode != "paper":
        raise ValueError(f"unknown mode {mode!r}")
    return _paper_vjp(M, B, dA, eps, eps_mul)


def moments_adjoint(dXtX, dXtY, x, y, r: int):
    """XtX_k = sum_{j in T_k} x_j x_j^T, XtY_k = sum_{j in T_k} x_j y_j^T.
    With G_j = sum_{k in T_j} dXtX_k and Gy_j = sum_{k in T_j} dXtY_k:
    dx_j = (G_j + G_j^T) x_j + Gy_j y_j and dy_j = Gy_j^T x_j."""
    G = window_sum(np.moveaxis(dXtX, (-2, -1), (0, 1)), r)       # [F,F,H,W]
    Gy = window_sum(np.moveaxis(dXtY, (-2, -1), (0, 1)), r)      # [F,C,H,W]
    dx = np.einsum("fghw,ghw->fhw", G + np.swapaxes(G, 0, 1), x)
    dx += np.einsum("fchw,chw->fhw", Gy, y)
    dy = np.einsum("fchw,fhw->chw", Gy, x)
    return dx, dy


def flr_backward(noisy, guides, grad_out, radius: int, eps: float, mode: str = "ridge",
                 eps_mul: float = 0.0, average: bool = True):
    """(d_noisy [C,H,W], d_guides [Q,H,W], d_eps, d_eps_mul) of
    L = sum(grad_out * flr_reference(noisy, guides, radius, eps, mode, eps_mul, average))."""
    y = np.asarray(noisy, dtype=np.float64)
    x = design_stack(guides)
    G = np.asarray(grad_out, dtype=np.float64)
    n, XtX, XtY = window_moments(y, guides, radius)
    nn = n[..., None, None]
    M, B = XtX / nn, XtY / nn
    A = solve_normalised(M, B, eps, mode, eps_mul)
    Abar = average_coefficients(A, radius) if average else A
    dAbar, dx = reconstruction_adjoint(Abar, x, G)
    dA = averaging_adjoint(dAbar, radius) if average else dAbar
    dM, dB, deps, dem = solve_vjp(M, B, dA, eps, mode, eps_mul)
    dxm, dy = moments_adjoint(dM / nn, dB / nn, x, y, radius)
    dx = dx + dxm
    return dy, dx[1:], deps, dem
