"""Pins of the FP64 FLR adjoint oracle (oracle/flr_adjoint.py), CPU only.

The adjoint is checked against things it does not compute itself:
* central finite differences of the forward oracle, element by element, for
  dL/d(noisy), dL/d(guides), dL/d(eps) and dL/d(eps_mul) in every regulariser
  mode, with and without coefficient averaging;
* exactness in the noisy input: for fixed guides the output is linear in the
  noisy image, so <G, F(y + d)> - <G, F(y)> = <dL/dy, d> holds to rounding
  for any d (no truncation error);
* a brute-force gradient: torch autograd (FP64, CPU) through explicit
  per-window normal equations built from the window's pixel rows;
* closed forms: r = 0 (output = noisy input) and a huge regulariser without
  averaging (output = window mean of the noisy input);
* planted mistakes in the adjoint must fail these pins.
"""
import numpy as np
import pytest

from oracle import flr_adjoint as adj
from oracle.flr_ref import flr_reference, window_count, window_sum
from synth import random_frame


def _rel(a, b):
    return np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300)


def _frame(H=5, W=6, Q=2, C=2, seed=1, offset=1.5):
    fr = random_frame(H, W, Q, C, seed=seed, offset=offset)
    rng = np.random.default_rng(seed + 100)
    return (fr["noisy"].astype(np.float64), fr["guides"].astype(np.float64),
            rng.standard_normal(fr["noisy"].shape))


def _fd(y, g, G, r, eps, mode, em, avg, h=1e-5):
    def L(yy, gg, e, m):
        return float(np.sum(G * flr_reference(yy, gg, r, e, mode, m, average=avg)))
    fdy = np.zeros_like(y)
    fdg = np.zeros_like(g)
    for idx in np.ndindex(y.shape):
        yp, ym = y.copy(), y.copy()
        yp[idx] += h
        ym[idx] -= h
        fdy[idx] = (L(yp, g, eps, em) - L(ym, g, eps, em)) / (2 * h)
    for idx in np.ndindex(g.shape):
        gp, gm = g.copy(), g.copy()
        gp[idx] += h
        gm[idx] -= h
        fdg[idx] = (L(y, gp, eps, em) - L(y, gm, eps, em)) / (2 * h)
    he = eps * 1e-4
    fde = (L(y, g, eps + he, em) - L(y, g, eps - he, em)) / (2 * he)
    fdm = 0.0
    if mode == "paper":
        fdm = (L(y, g, eps, em + 1e-5) - L(y, g, eps, em - 1e-5)) / 2e-5
    return fdy, fdg, fde, fdm


FD_CASES = [
    dict(mode="ridge", avg=True, eps=1e-2, em=0.0, r=2),
    dict(mode="ridge", avg=False, eps=1e-2, em=0.0, r=2),
    dict(mode="ridge", avg=True, eps=3e-3, em=0.0, r=1, Q=3, C=1, W=7),
    dict(mode="raw", avg=True, eps=1e-2, em=0.0, r=1),
    dict(mode="paper", avg=True, eps=1e-2, em=0.3, r=2),
    dict(mode="paper", avg=False, eps=5e-2, em=0.2, r=1),
    dict(mode="paper", avg=True, eps=2e-2, em=0.0, r=3, H=4, W=9),
]


def _fd_ok(case, tol=1e-7) -> bool:
    c = dict(case)
    mode, avg, eps, em, r = c.pop("mode"), c.pop("avg"), c.pop("eps"), c.pop("em"), c.pop("r")
    y, g, G = _frame(**c)
    dy, dg, de, dm = adj.flr_backward(y, g, G, r, eps, mode, em, avg)
    fdy, fdg, fde, fdm = _fd(y, g, G, r, eps, mode, em, avg)
    ok = _rel(dy, fdy) < tol and _rel(dg, fdg) < tol
    ok &= abs(de - fde) <= tol * max(abs(fde), 1.0)
    ok &= abs(dm - fdm) <= tol * max(abs(fdm), 1.0)
    return bool(ok)


@pytest.mark.parametrize("case", FD_CASES, ids=lambda c: f"{c['mode']}-avg{int(c['avg'])}-r{c['r']}")
def test_adjoint_matches_finite_differences(case):
    assert _fd_ok(case)


@pytest.mark.parametrize("mode,avg", [("ridge", True), ("ridge", False), ("paper", True)])
def test_noisy_gradient_exact_by_linearity(mode, avg):
    y, g, G = _frame(H=12, W=13, Q=3, C=2, seed=4)
    r, eps, em = 3, 1e-2, 0.1 if mode == "paper" else 0.0
    dy, _, _, _ = adj.flr_backward(y, g, G, r, eps, mode, em, avg)
    d = np.random.default_rng(9).standard_normal(y.shape) * 3.0
    lhs = np.sum(G * (flr_reference(y + d, g, r, eps, mode, em, average=avg)
                      - flr_reference(y, g, r, eps, mode, em, average=avg)))
    rhs = np.sum(dy * d)
    assert abs(lhs - rhs) <= 1e-10 * np.sum(np.abs(dy * d))


def _brute_torch_loss(torch, y, g, G, r, eps, avg):
    """L = <G, out> with out from explicit per-window ridge normal equations
    (bias unpenalised), built row by row from the window's pixels."""
    C, H, W = y.shape
    Q = g.shape[0]
    pen = torch.eye(Q + 1, dtype=torch.float64)
    pen[0, 0] = 0.0
    A = {}
    for i in range(H):
        for j in range(W):
            rows = [(a, b) for a in range(max(0, i - r), min(H, i + r + 1))
                    for b in range(max(0, j - r), min(W, j + r + 1))]
            X = torch.stack([torch.cat([torch.ones(1, dtype=torch.float64), g[:, a, b]])
                             for a, b in rows])
            Y = torch.stack([y[:, a, b] for a, b in rows])
            n = float(len(rows))
            A[i, j] = torch.linalg.solve(X.T @ X / n + eps * pen, X.T @ Y / n)
    L = 0.0
    for i in range(H):
        for j in range(W):
            if avg:
                ks = [A[a, b] for a in range(max(0, i - r), min(H, i + r + 1))
                      for b in range(max(0, j - r), min(W, j + r + 1))]
                Ab = torch.stack(ks).mean(0)
            else:
                Ab = A[i, j]
            x = torch.cat([torch.ones(1, dtype=torch.float64), g[:, i, j]])
            L = L + torch.dot(G[:, i, j], x @ Ab)
    return L


@pytest.mark.parametrize("avg,r,Q", [(True, 2, 2), (False, 2, 2), (True, 1, 3)])
def test_adjoint_matches_brute_force_autograd(avg, r, Q):
    torch = pytest.importorskip("torch")
    y, g, G = _frame(H=6, W=7, Q=Q, C=2, seed=5)
    eps = 1e-2
    ty = torch.tensor(y, requires_grad=True)
    tg = torch.tensor(g, requires_grad=True)
    te = torch.tensor(eps, dtype=torch.float64, requires_grad=True)
    L = _brute_torch_loss(torch, ty, tg, torch.tensor(G), r, te, avg)
    gy, gg, ge = torch.autograd.grad(L, (ty, tg, te))
    dy, dg, de, _ = adj.flr_backward(y, g, G, r, eps, "ridge", 0.0, avg)
    assert _rel(dy, gy.numpy()) < 1e-9
    assert _rel(dg, gg.numpy()) < 1e-9
    assert abs(de - ge.item()) <= 1e-9 * max(abs(ge.item()), 1.0)


@pytest.mark.parametrize("mode,eps,em", [("ridge", 1e-3, 0.0), ("paper", 1e-2, 0.1)])
def test_gradient_check_instance_32x32(mode, eps, em):
    """The training workload's named gradient check: a 32x32 frame with 4
    guides plus the constant (5 features), radius 3, FP64. dL/d(noisy) in
    full by linearity, dL/d(guides) by central differences on 160 seeded
    entries (borders, corners and interior), dL/d(eps) and, for the
    Appendix regulariser, dL/d(eps') by central differences."""
    from synth import make_config
    fr = make_config(0, h=32, w=32)
    y = fr["noisy"].astype(np.float32).astype(np.float64)
    g = fr["guides"].astype(np.float32).astype(np.float64)
    assert g.shape == (4, 32, 32)
    G = np.random.default_rng(33).standard_normal(y.shape)
    r = 3
    dy, dg, de, dm = adj.flr_backward(y, g, G, r, eps, mode, em, True)

    def L(yy, gg, e=eps, m=em):
        return float(np.sum(G * flr_reference(yy, gg, r, e, mode, m, average=True)))

    d = np.random.default_rng(34).standard_normal(y.shape)
    lhs = L(y + d, g) - L(y, g)
    assert abs(lhs - np.sum(dy * d)) <= 1e-10 * np.sum(np.abs(dy * d))
    rng = np.random.default_rng(35)
    idx = [tuple(rng.integers(0, s) for s in g.shape) for _ in range(150)]
    idx += [(q, a, b) for q in range(4) for a, b in [(0, 0), (31, 31), (0, 31)]][:10]
    h = 1e-5
    scale = np.max(np.abs(dg))
    for i in idx:
        gp, gm = g.copy(), g.copy()
        gp[i] += h
        gm[i] -= h
        fd = (L(y, gp) - L(y, gm)) / (2 * h)
        assert abs(fd - dg[i]) <= 1e-6 * scale, (i, fd, dg[i])
    he = eps * 1e-4
    fde = (L(y, g, eps + he) - L(y, g, eps - he)) / (2 * he)
    assert abs(de - fde) <= 1e-6 * max(abs(fde), 1.0)
    if mode == "paper":
        fdm = (L(y, g, eps, em + 1e-5) - L(y, g, eps, em - 1e-5)) / 2e-5
        assert abs(dm - fdm) <= 1e-6 * max(abs(fdm), 1.0)


def test_radius_zero_is_identity():
    """r = 0: each window is one pixel, W = V = 0, a = 0, out = noisy."""
    y, g, G = _frame(H=4, W=5, Q=2, C=3, seed=6)
    for mode, em in (("ridge", 0.0), ("paper", 0.2)):
        for avg in (True, False):
            dy, dg, de, dm = adj.flr_backward(y, g, G, 0, 1e-2, mode, em, avg)
            assert _rel(dy, G) < 1e-12
            assert np.max(np.abs(dg)) < 1e-10 and abs(de) < 1e-10 and abs(dm) < 1e-10


def test_huge_regulariser_gives_window_mean_adjoint():
    """eps -> infinity without averaging: a -> 0, out -> window mean of y, so
    dL/dy -> sum over windows containing j of G_k / n_k; dL/dg -> 0."""
    y, g, G = _frame(H=7, W=8, Q=2, C=2, seed=7)
    r = 2
    dy, dg, _, _ = adj.flr_backward(y, g, G, r, 1e12, "ridge", 0.0, False)
    want = window_sum(G / window_count(7, 8, r), r)
    assert _rel(dy, want) < 1e-9
    assert np.max(np.abs(dg)) < 1e-9 * np.max(np.abs(want))


# --- planted mistakes -------------------------------------------------------

def _battery() -> bool:
    return all(_fd_ok(c, tol=1e-6) for c in (FD_CASES[0], FD_CASES[1], FD_CASES[4]))


def _moments_no_transpose(dXtX, dXtY, x, y, r):
    # forgets that x enters x x^T twice: dx = G x instead of (G + G^T) x
    G = window_sum(np.moveaxis(dXtX, (-2, -1), (0, 1)), r)
    Gy = window_sum(np.moveaxis(dXtY, (-2, -1), (0, 1)), r)
    dx = np.einsum("fghw,ghw->fhw", G, x) + np.einsum("fchw,chw->fhw", Gy, y)
    return dx, np.einsum("fchw,fhw->chw", Gy, x)


def _reconstruction_no_direct(Abar, x, G, _orig=adj.reconstruction_adjoint):
    dAbar, dx = _orig(Abar, x, G)
    return dAbar, np.zeros_like(dx)


def _averaging_no_count(dAbar, r):
    t = np.moveaxis(dAbar, (0, 1), (2, 3))
    return np.moveaxis(window_sum(t, r), (2, 3), (0, 1))


def _solve_sign_slip(M, B, dA, eps, mode="ridge", eps_mul=0.0, _orig=adj.solve_vjp):
    dM, dB, de, dm = _orig(M, B, dA, eps, mode, eps_mul)
    return -dM, dB, -de, -dm


def _solve_no_inverse(M, B, dA, eps, mode="ridge", eps_mul=0.0, _orig=adj.solve_vjp):
    # passes dA straight to dB, forgetting the K^-1 of A = K^-1 B
    dM, dB, de, dm = _orig(M, B, dA, eps, mode, eps_mul)
    return dM, np.array(dA, dtype=np.float64), de, dm


def _paper_eps_once(M, B, dA, eps, em, _orig=adj._paper_vjp):
    # forgets that eps also enters W^ (counts only the eps of C^ + eps I)
    dM, dB, de, dm = _orig(M, B, dA, eps, em)
    return dM, dB, de - float(np.sum(np.trace(dM[..., 1:, 1:], axis1=-2, axis2=-1))), dm


def _paper_no_diag_mu(M, B, dA, eps, em, _orig=adj._paper_vjp):
    # drops the eps' diag(mu o mu) term from dL/dmu
    dM, dB, de, dm = _orig(M, B, dA, eps, em)
    dM = dM.copy()
    mu = M[..., 0, 1:]
    dM[..., 0, 1:] -= em * 2.0 * np.diagonal(dM[..., 1:, 1:], axis1=-2, axis2=-1) * mu
    return dM, dB, de, dm


MUTATIONS = [
    ("moments_adjoint", _moments_no_transpose),
    ("reconstruction_adjoint", _reconstruction_no_direct),
    ("averaging_adjoint", _averaging_no_count),
    ("solve_vjp", _solve_sign_slip),
    ("solve_vjp", _solve_no_inverse),
    ("_paper_vjp", _paper_eps_once),
    ("_paper_vjp", _paper_no_diag_mu),
]


def test_unmutated_adjoint_passes_battery():
    assert _battery()


@pytest.mark.parametrize("name,fn", MUTATIONS, ids=[f"{n}-{f.__name__}" for n, f in MUTATIONS])
def test_planted_adjoint_mistake_is_caught(monkeypatch, name, fn):
    monkeypatch.setattr(adj, name, fn)
    assert not _battery()
