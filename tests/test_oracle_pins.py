"""Pins for the FP64 oracle: brute force, exact arithmetic, closed forms and invariants.

Each test ties the oracle to something other than itself: explicit window
loops, an SVD least-squares solve, exact rational arithmetic, the textbook
single-guide guided filter (box sums by ``scipy.signal.convolve2d``), global
least squares when the window covers the image, and invariances that the
least-squares definition fixes (Sec. 3.1-3.2 and the Appendix).
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy.signal import convolve2d

from oracle import brute
from oracle import flr_ref as ref
from synth import make_config, random_frame, small_integer_frame


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


# --------------------------------------------------------------------------
# Moments: window sums of outer products equal the explicit per-window X^T X.

@pytest.mark.parametrize("h,w", [(1, 1), (1, 6), (5, 1), (5, 7), (7, 13), (13, 5)])
@pytest.mark.parametrize("r", [0, 1, 2, 3, 20])
def test_moments_match_explicit_windows_exactly(h, w, r):
    fr = small_integer_frame(h, w, q=3, c=2, seed=h * 100 + w * 7 + r)
    n, XtX, XtY = ref.window_moments(fr["noisy"], fr["guides"], r)
    nb, XtXb, XtYb = brute.brute_moments(fr["noisy"], fr["guides"], r)
    # integer data: sums are exact in float64 on both routes
    assert np.array_equal(n, nb)
    assert np.array_equal(XtX, XtXb)
    assert np.array_equal(XtY, XtYb)


def test_window_count_closed_form_interior_and_corner():
    n = ref.window_count(40, 50, 8)
    assert n[20, 25] == 17 * 17          # interior: full (2r+1)^2 window
    assert n[0, 0] == 9 * 9              # corner: r+1 by r+1
    assert n[0, 25] == 9 * 17            # top edge
    assert n[39, 49] == 9 * 9


# --------------------------------------------------------------------------
# Solve: ridge coefficients against per-window lstsq on the stacked system.

@pytest.mark.parametrize("h,w,r,q,c", [(5, 7, 1, 1, 1), (7, 6, 2, 2, 3), (9, 9, 3, 4, 1),
                                       (6, 11, 2, 4, 3), (2, 3, 5, 2, 1)])
@pytest.mark.parametrize("average", [False, True])
def test_ridge_matches_bruteforce_lstsq(h, w, r, q, c, average):
    fr = random_frame(h, w, q, c, seed=11 * h + w + r, smooth=0.0)
    eps = 1e-2
    out, A = ref.flr_reference(fr["noisy"], fr["guides"], r, eps, "ridge", average=average,
                               return_coeffs=True)
    outb, Ab = brute.ridge_brute(fr["noisy"], fr["guides"], r, eps, average=average)
    assert _rel(A, Ab) < 1e-9
    assert _rel(out, outb) < 1e-10


def _exact_solve(M, b):
    """Gauss-Jordan elimination in exact rationals."""
    n = len(M)
    aug = [list(M[i]) + list(b[i]) for i in range(n)]
    m = len(b[0])
    for col in range(n):
        piv = next(i for i in range(col, n) if aug[i][col] != 0)
        aug[col], aug[piv] = aug[piv], aug[col]
        pv = aug[col][col]
        aug[col] = [v / pv for v in aug[col]]
        for i in range(n):
            if i != col and aug[i][col] != 0:
                f = aug[i][col]
                aug[i] = [vi - f * vc for vi, vc in zip(aug[i], aug[col])]
    return [[aug[i][n + j] for j in range(m)] for i in range(n)]


def test_exact_rational_least_squares_tiny():
    """Exact rational arithmetic from the least-squares definition (no rounding at all)."""
    H, W, Q, C, r = 4, 5, 2, 2, 1
    fr = small_integer_frame(H, W, Q, C, seed=5)
    g = fr["guides"].astype(int)
    y = fr["noisy"].astype(int)
    eps = Fraction(1, 50)
    F = Q + 1
    A = {}
    for i in range(H):
        for j in range(W):
            rows = [(ii, jj) for ii in range(i - r, i + r + 1) for jj in range(j - r, j + r + 1)
                    if 0 <= ii < H and 0 <= jj < W]
            nk = len(rows)
            X = [[Fraction(1)] + [Fraction(int(g[q, ii, jj])) for q in range(Q)] for ii, jj in rows]
            Y = [[Fraction(int(y[cc, ii, jj])) for cc in range(C)] for ii, jj in rows]
            M = [[sum(X[t][a] * X[t][b] for t in range(nk)) / nk + (eps if (a == b and a > 0) else 0)
                  for b in range(F)] for a in range(F)]
            B = [[sum(X[t][a] * Y[t][cc] for t in range(nk)) / nk for cc in range(C)]
                 for a in range(F)]
            A[i, j] = _exact_solve(M, B)
    out = np.zeros((C, H, W))
    for i in range(H):
        for j in range(W):
            ks = [(ii, jj) for ii in range(i - r, i + r + 1) for jj in range(j - r, j + r + 1)
                  if 0 <= ii < H and 0 <= jj < W]
            x = [Fraction(1)] + [Fraction(int(g[q, i, j])) for q in range(Q)]
            for cc in range(C):
                s = sum(sum(x[f] * A[k][f][cc] for f in range(F)) for k in ks) / len(ks)
                out[cc, i, j] = float(s)
    got = ref.flr_reference(fr["noisy"], fr["guides"], r, float(eps), "ridge", average=True)
    assert _rel(got, out) < 1e-12


# A 1 x 3 frame worked by hand from Sec. 3.1's closed form (ridge on the
# centred system with eps added in covariance scale, reading c4): guide
# g = (0, 1, 2), channel y = (1, 2, 4), r = 1, eps = 1/2. The clipped
# windows are {0, 1}, {0, 1, 2}, {1, 2}; their means, variances and
# covariances give slopes a = V / (W + eps):
#   {0, 1}:    mu 1/2, nu 3/2, W 1/4, V 1/4 -> a 1/3, b = nu - a mu = 4/3
#   {0, 1, 2}: mu 1,   nu 7/3, W 2/3, V 1   -> a 6/7, b = 31/21
#   {1, 2}:    mu 3/2, nu 3,   W 1/4, V 1/2 -> a 2/3, b = 2
# Per-pixel models give out = b + a g = (4/3, 7/3, 10/3). With the models
# averaged over each pixel's window (reading c2): abar = (25/42, 13/21,
# 16/21), bbar = (59/42, 101/63, 73/42), out = (59/42, 20/9, 137/42).
HAND_1X3 = dict(g=[0.0, 1.0, 2.0], y=[1.0, 2.0, 4.0], r=1, eps=0.5,
                plain=[4 / 3, 7 / 3, 10 / 3], averaged=[59 / 42, 20 / 9, 137 / 42])


@pytest.mark.parametrize("average", [False, True])
def test_hand_worked_1x3(average):
    h = HAND_1X3
    g = np.array(h["g"]).reshape(1, 1, 3)
    y = np.array(h["y"]).reshape(1, 1, 3)
    got = ref.flr_reference(y, g, h["r"], h["eps"], "ridge", average=average)
    want = np.array(h["averaged" if average else "plain"]).reshape(1, 1, 3)
    assert np.max(np.abs(got - want)) < 1e-14


# --------------------------------------------------------------------------
# Closed forms and special cases.

def _box_sum_conv(img, r):
    return convolve2d(img, np.ones((2 * r + 1, 2 * r + 1)), mode="same", boundary="fill")


@pytest.mark.parametrize("eps", [1e-3, 0.1])
def test_single_guide_equals_textbook_guided_filter(eps):
    """Q = 1, averaged: the guided filter of He et al. (Sec. 2) with clipped box means."""
    fr = random_frame(23, 31, 1, 1, seed=3, smooth=2.0)
    I = fr["guides"][0].astype(np.float64)
    p = fr["noisy"][0].astype(np.float64)
    r = 3
    N = _box_sum_conv(np.ones_like(I), r)
    mean = lambda z: _box_sum_conv(z, r) / N
    mI, mp = mean(I), mean(p)
    var = mean(I * I) - mI * mI
    cov = mean(I * p) - mI * mp
    a = cov / (var + eps)
    b = mp - a * mI
    q = mean(a) * I + mean(b)
    got = ref.flr_reference(fr["noisy"], fr["guides"], r, eps, "ridge", average=True)[0]
    assert _rel(got, q) < 1e-11


@pytest.mark.parametrize("mode", ["ridge", "paper"])
def test_radius_zero_returns_input(mode):
    fr = random_frame(9, 8, 3, 2, seed=4)
    out = ref.flr_reference(fr["noisy"], fr["guides"], 0, 1e-3, mode, average=True)
    # n = 1, zero covariance: a = 0 and b = y, up to the solver's rounding
    assert _rel(out, fr["noisy"]) < 1e-13


@pytest.mark.parametrize("average", [False, True])
def test_window_covering_image_is_one_global_fit(average):
    H, W, Q, C, r = 6, 9, 3, 2, 8
    fr = random_frame(H, W, Q, C, seed=8)
    eps = 1e-2
    X = np.concatenate([np.ones((H * W, 1)), fr["guides"].reshape(Q, -1).T.astype(np.float64)], 1)
    Y = fr["noisy"].reshape(C, -1).T.astype(np.float64)
    pen = np.hstack([np.zeros((Q, 1)), np.sqrt(H * W * eps) * np.eye(Q)])
    A = np.linalg.lstsq(np.vstack([X, pen]), np.vstack([Y, np.zeros((Q, C))]), rcond=None)[0]
    want = (X @ A).T.reshape(C, H, W)
    got = ref.flr_reference(fr["noisy"], fr["guides"], r, eps, "ridge", average=average)
    assert _rel(got, want) < 1e-10


@pytest.mark.parametrize("mode", ["ridge", "paper"])
@pytest.mark.parametrize("average", [False, True])
def test_linear_input_reproduced_as_eps_to_zero(mode, average):
    fr = random_frame(14, 17, 3, 2, seed=12)
    g = fr["guides"].astype(np.float64)
    rng = np.random.default_rng(0)
    alpha = rng.normal(size=(3, 2))
    beta = rng.normal(size=2)
    y = np.einsum("qhw,qc->chw", g, alpha) + beta[:, None, None]
    out = ref.flr_reference(y, g, 2, 1e-12, mode, average=average)
    assert _rel(out, y) < 1e-8


@pytest.mark.parametrize("mode,eps_mul", [("ridge", 0.0), ("paper", 0.0), ("paper", 0.3)])
@pytest.mark.parametrize("average", [False, True])
def test_constant_input_maps_to_constant(mode, eps_mul, average):
    fr = random_frame(11, 13, 4, 1, seed=2)
    y = np.full((2, 11, 13), 3.25)
    out = ref.flr_reference(y, fr["guides"], 3, 0.05, mode, eps_mul=eps_mul, average=average)
    assert np.max(np.abs(out - 3.25)) < 1e-12


def test_large_eps_tends_to_box_mean():
    fr = random_frame(12, 10, 3, 2, seed=6)
    y = fr["noisy"].astype(np.float64)
    r = 2
    n = ref.window_count(12, 10, r)
    m1 = ref.window_sum(y, r) / n
    m2 = ref.window_sum(m1, r) / n
    out0 = ref.flr_reference(fr["noisy"], fr["guides"], r, 1e12, "ridge", average=False)
    out1 = ref.flr_reference(fr["noisy"], fr["guides"], r, 1e12, "ridge", average=True)
    assert _rel(out0, m1) < 1e-9
    assert _rel(out1, m2) < 1e-9


def test_raw_reading_breaks_constant_invariant():
    """Eq. tikhonov as written penalises the bias: constant input is shrunk."""
    fr = random_frame(9, 9, 2, 1, seed=1)
    y = np.full((1, 9, 9), 2.0)
    out = ref.flr_reference(y, fr["guides"], 2, 0.5, "raw", average=False)
    assert np.max(np.abs(out - 2.0)) > 1e-3


def test_raw_matches_bruteforce_penalising_all_coefficients():
    fr = random_frame(6, 7, 2, 1, seed=9)
    r, eps = 1, 0.2
    _, A = ref.flr_reference(fr["noisy"], fr["guides"], r, eps, "raw", average=False,
                             return_coeffs=True)
    for (i, j) in [(0, 0), (3, 4), (5, 6)]:
        X, Y = brute.window_matrices(fr["noisy"], fr["guides"], r, i, j)
        nk = X.shape[0]
        Xa = np.vstack([X, np.sqrt(nk * eps) * np.eye(3)])
        Ya = np.vstack([Y, np.zeros((3, 1))])
        want = np.linalg.lstsq(Xa, Ya, rcond=None)[0]
        assert _rel(A[i, j], want) < 1e-10


# --------------------------------------------------------------------------
# Invariances fixed by the least-squares definition.

@pytest.mark.parametrize("average", [False, True])
def test_affine_equivariance_in_y(average):
    fr = random_frame(10, 12, 3, 2, seed=21)
    r, eps = 2, 1e-2
    o1 = ref.flr_reference(fr["noisy"], fr["guides"], r, eps, average=average)
    o2 = ref.flr_reference(2.5 * fr["noisy"].astype(np.float64) - 0.75, fr["guides"], r, eps,
                           average=average)
    assert _rel(o2, 2.5 * o1 - 0.75) < 1e-12


@pytest.mark.parametrize("mode", ["ridge", "paper"])
def test_guide_shift_invariance(mode):
    fr = random_frame(10, 9, 3, 1, seed=22)
    g2 = fr["guides"].astype(np.float64) + np.array([5.0, -3.0, 100.0])[:, None, None]
    o1 = ref.flr_reference(fr["noisy"], fr["guides"], 2, 1e-2, mode)
    o2 = ref.flr_reference(fr["noisy"], g2, 2, 1e-2, mode)
    assert _rel(o1, o2) < 1e-9


def test_guide_permutation_invariance():
    fr = random_frame(9, 11, 4, 2, seed=23)
    perm = [2, 0, 3, 1]
    o1 = ref.flr_reference(fr["noisy"], fr["guides"], 2, 1e-2)
    o2 = ref.flr_reference(fr["noisy"], fr["guides"][perm], 2, 1e-2)
    assert _rel(o1, o2) < 1e-12


@pytest.mark.parametrize("op", ["flipud", "fliplr", "transpose"])
def test_flip_and_transpose_equivariance(op):
    fr = random_frame(8, 13, 2, 2, seed=24)
    f = {"flipud": lambda a: a[..., ::-1, :], "fliplr": lambda a: a[..., :, ::-1],
         "transpose": lambda a: np.swapaxes(a, -1, -2)}[op]
    o1 = ref.flr_reference(fr["noisy"], fr["guides"], 3, 1e-2)
    o2 = ref.flr_reference(f(fr["noisy"]), f(fr["guides"]), 3, 1e-2)
    assert _rel(f(o1), o2) < 1e-12


# --------------------------------------------------------------------------
# Second formulations of the solve.

def test_centred_system_equals_bordered_system():
    """(W + eps I) a = V, b = nu - a^T mu equals the bordered (Q+1) solve."""
    fr = make_config(0, h=24, w=20)
    r, eps = 3, 1e-3
    _, A = ref.flr_reference(fr["noisy"], fr["guides"], r, eps, average=False, return_coeffs=True)
    P = ref.central_moment_planes(fr["noisy"], fr["guides"], r)
    Q, C = 4, 1
    mu = np.moveaxis(P[1:1 + Q], 0, -1)
    nu = np.moveaxis(P[1 + Q:1 + Q + C], 0, -1)
    k = 1 + Q + C
    Wc = np.zeros(mu.shape[:2] + (Q, Q))
    for p in range(Q):
        for q in range(p, Q):
            Wc[..., p, q] = Wc[..., q, p] = P[k]
            k += 1
    Vc = np.moveaxis(P[k:], 0, -1).reshape(mu.shape[:2] + (Q, C))
    a = np.linalg.solve(Wc + eps * np.eye(Q), Vc)
    b = nu - np.einsum("hwq,hwqc->hwc", mu, a)
    assert _rel(A[..., 1:, :], a) < 1e-9
    assert _rel(A[..., 0, :], b) < 1e-10


@pytest.mark.parametrize("eps,eps_mul", [(1e-3, 0.0), (1e-2, 0.2), (1e-4, 1.0)])
def test_paper_literal_equals_compact_system(eps, eps_mul):
    """Appendix normalisation = solve (W_hat + eps diag W_hat) a = V (derived algebraically)."""
    fr = random_frame(9, 10, 3, 2, seed=31, offset=2.0)
    r = 2
    n, XtX, XtY = ref.window_moments(fr["noisy"], fr["guides"], r)
    _, A = ref.flr_reference(fr["noisy"], fr["guides"], r, eps, "paper", eps_mul=eps_mul,
                             average=False, return_coeffs=True)
    nn = n[..., None, None]
    M, B = XtX / nn, XtY / nn
    mu = M[..., 0, 1:]
    nu = B[..., 0, :]
    mumu = mu[..., :, None] * mu[..., None, :]
    Wc = M[..., 1:, 1:] - mumu
    Vc = B[..., 1:, :] - mu[..., :, None] * nu[..., None, :]
    Q = 3
    What = Wc + eps_mul * (mumu + np.eye(Q) * (mu * mu)[..., None, :]) + eps * np.eye(Q)
    Hm = What + eps * np.eye(Q) * np.diagonal(What, axis1=-2, axis2=-1)[..., None, :]
    a = np.linalg.solve(Hm, Vc)
    b = nu - np.einsum("hwq,hwqc->hwc", mu, a)
    assert _rel(A[..., 1:, :], a) < 1e-9
    assert _rel(A[..., 0, :], b) < 1e-9


def test_paper_with_zero_regularisers_equals_unregularised_ridge():
    fr = random_frame(10, 10, 2, 1, seed=33)
    o1 = ref.flr_reference(fr["noisy"], fr["guides"], 3, 0.0, "paper", eps_mul=0.0)
    o2 = ref.flr_reference(fr["noisy"], fr["guides"], 3, 0.0, "ridge")
    assert _rel(o1, o2) < 1e-9


# --------------------------------------------------------------------------
# Plane layouts and the block evaluator.

def test_plane_round_trips():
    fr = random_frame(7, 8, 3, 2, seed=40)
    P = ref.central_moment_planes(fr["noisy"], fr["guides"], 2)
    assert P.shape[0] == 1 + 3 + 2 + 6 + 6
    n, M, B = ref.moments_from_central_planes(P, 3, 2)
    n2, XtX, XtY = ref.window_moments(fr["noisy"], fr["guides"], 2)
    assert np.array_equal(n, n2)
    assert _rel(M, XtX / n2[..., None, None]) < 1e-13
    assert _rel(B, XtY / n2[..., None, None]) < 1e-13
    _, A = ref.flr_reference(fr["noisy"], fr["guides"], 2, 1e-2, return_coeffs=True)
    assert np.array_equal(ref.coefficients_from_planes(ref.coefficient_planes(A), 3, 2), A)


def test_block_evaluator_matches_full_frame():
    fr = make_config(0, h=70, w=64)
    r, eps = 4, 1e-3
    full = ref.flr_reference(fr["noisy"], fr["guides"], r, eps)
    for (y0, y1, x0, x1) in [(0, 10, 0, 12), (30, 41, 20, 33), (60, 70, 50, 64)]:
        blk = ref.flr_reference_block(fr["noisy"], fr["guides"], r, eps, y0, y1, x0, x1)
        assert _rel(blk, full[:, y0:y1, x0:x1]) < 1e-12
