"""Brute-force per-window least squares, for pinning the FP64 oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/flr_ref.py``). Tiny images only.

For every pixel k it builds the window matrices X_k (leading column of ones,
one column per guide; Sec. 3.1, Eq. matX) and Y_k (Eq. matY) pixel by pixel
with explicit loops, and solves the regularised least-squares problem by
``numpy.linalg.lstsq`` (an SVD) on the stacked system

    [ X_k                       ]       [ Y_k ]
    [ sqrt(n_k eps) [0 | I_Q]   ] A  ~  [  0  ]

which minimises ||X_k A - Y_k||^2 + n_k eps ||a||^2, the ridge reading of
Eq. tikhonov in covariance scale with the bias left unpenalised. This is a
different numerical route from the oracle's normal equations.
"""
from __future__ import annotations

import numpy as np

__all__ = ["window_matrices", "ridge_brute", "brute_moments"]


def window_matrices(noisy, guides, r: int, i: int, j: int):
    """X_k [N,F] and Y_k [N,C] for the clipped window centred at (i, j)."""
    Q, H, W = guides.shape
    C = noisy.shape[0]
    rows_x, rows_y = [], []
    for ii in range(i - r, i + r + 1):
        for jj in range(j - r, j + r + 1):
            if 0 <= ii < H and 0 <= jj < W:
                rows_x.append([1.0] + [float(guides[q, ii, jj]) for q in range(Q)])
                rows_y.append([float(noisy[c, ii, jj]) for c in range(C)])
    return np.array(rows_x, dtype=np.float64), np.array(rows_y, dtype=np.float64)


def brute_moments(noisy, guides, r: int):
    """X_k^T X_k [H,W,F,F] and X_k^T Y_k [H,W,F,C] by explicit window loops."""
    Q, H, W = guides.shape
    C = noisy.shape[0]
    F = Q + 1
    XtX = np.zeros((H, W, F, F))
    XtY = np.zeros((H, W, F, C))
    n = np.zeros((H, W))
    for i in range(H):
        for j in range(W):
            X, Y = window_matrices(noisy, guides, r, i, j)
            XtX[i, j] = X.T @ X
            XtY[i, j] = X.T @ Y
            n[i, j] = X.shape[0]
    return n, XtX, XtY


def ridge_brute(noisy, guides, r: int, eps: float, average: bool = True):
    """Denoised [C,H,W] and unaveraged coefficients [H,W,F,C] by brute force."""
    Q, H, W = guides.shape
    C = noisy.shape[0]
    F = Q + 1
    A = np.zeros((H, W, F, C))
    for i in range(H):
        for j in range(W):
            X, Y = window_matrices(noisy, guides, r, i, j)
            nk = X.shape[0]
            pen = np.zeros((Q, F))
            pen[:, 1:] = np.sqrt(nk * eps) * np.eye(Q)
            Xa = np.vstack([X, pen])
            Ya = np.vstack([Y, np.zeros((Q, C))])
            A[i, j] = np.linalg.lstsq(Xa, Ya, rcond=None)[0]
    out = np.zeros((C, H, W))
    for i in range(H):
        for j in range(W):
            x = np.array([1.0] + [float(guides[q, i, j]) for q in range(Q)])
            if average:
                acc = np.zeros((F, C))
                cnt = 0
                for ii in range(i - r, i + r + 1):
                    for jj in range(j - r, j + r + 1):
                        if 0 <= ii < H and 0 <= jj < W:
                            acc += A[ii, jj]
                            cnt += 1
                Ak = acc / cnt
            else:
                Ak = A[i, j]
            out[:, i, j] = x @ Ak
    return out, A
