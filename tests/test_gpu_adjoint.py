"""GPU parity of the FLR adjoint (flr_denoise_backward) and its autograd wrapper.

The GPU adjoint is compared element by element with the FP64 adjoint oracle
(oracle/flr_adjoint.py, itself pinned to finite differences and a
brute-force gradient) on the same FP32 inputs, with eps and eps_mul rounded
to FP32 as the C ABI carries them. Every step of the GPU adjoint is FP64
(moments from FP64 window sums of anchored products, FP64 fields and window
sums); the outputs are FP32. Tolerance: max |got - ref| / max(|ref|, 1e-3
rms(ref)) <= 1e-6 (output rounding is 6e-8); the regulariser gradients,
sums over all pixels in FP64, within 1e-8 relative.

At 1080p the oracle runs on crops: dL/d(guides) and dL/d(noisy) at pixel j
depend on dL/d(out) within 2r of j and on the inputs within 4r (moments of
windows within r of the pixels whose averaged model uses j), so crops with a
4r margin reproduce the full-frame gradient in their interior.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2410_11625_amd as flr  # noqa: E402
from oracle import flr_adjoint  # noqa: E402
from synth import make_config, random_frame  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-6


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(_dev())


def _rel(got, want):
    rms = max(float(np.sqrt(np.mean(np.asarray(want, np.float64) ** 2))), 1e-30)
    return float(np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-3 * rms)))


def _f32(x):
    return float(np.float32(x))


def _frame(case):
    H, W, Q, C = case["H"], case["W"], case["Q"], case["C"]
    if "config" in case:
        fr = make_config(case["config"], h=H, w=W)
        g = fr["guides"][:Q]
        y = fr["noisy"][:C]
    else:
        fr = random_frame(H, W, Q, C, seed=case.get("seed", 3), smooth=1.5,
                          offset=case.get("offset", 0.0))
        g, y = fr["guides"], fr["noisy"]
    G = np.random.default_rng(case.get("seed", 3) + 50).standard_normal((C, H, W))
    return (np.asarray(y, np.float32), np.asarray(g, np.float32), G.astype(np.float32))


CASES = [
    dict(H=256, W=256, Q=4, C=1, r=8, config=0),
    # the training workload's gradient-check instance: 32x32, 4 guides + 1, r 3
    dict(H=32, W=32, Q=4, C=1, r=3, config=0),
    dict(H=32, W=32, Q=4, C=1, r=3, config=0, mode="paper", eps=1e-2, eps_mul=0.1),
    dict(H=70, W=300, Q=8, C=3, r=8, config=1),
    dict(H=50, W=270, Q=8, C=3, r=8, config=1, average=False),
    dict(H=33, W=131, Q=3, C=2, r=3, mode="paper", eps=1e-2, eps_mul=0.2, offset=2.0),
    dict(H=40, W=200, Q=12, C=3, r=8, seed=7),
    dict(H=1, W=300, Q=2, C=1, r=2),
    dict(H=300, W=1, Q=1, C=2, r=3),
    dict(H=9, W=11, Q=2, C=1, r=20),
    dict(H=66, W=70, Q=4, C=4, r=32, mode="paper", eps=1e-3, eps_mul=0.05),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(
    f"{k}{c[k]}" for k in ("H", "W", "Q", "C", "r") ) + ("-" + c.get("mode", "ridge"))
    + ("-noavg" if c.get("average") is False else ""))
def test_backward_matches_oracle(case):
    y, g, G = _frame(case)
    r, eps, em = case["r"], case.get("eps", 1e-3), case.get("eps_mul", 0.0)
    mode, avg = case.get("mode", "ridge"), case.get("average", True)
    gy, gg, gr = flr.denoise_backward(_t(y), _t(g), _t(G), radius=r, eps=eps, mode=mode,
                                      eps_mul=em, average=avg)
    torch.cuda.synchronize()
    ry, rg, re, rm = flr_adjoint.flr_backward(y, g, G, r, _f32(eps), mode, _f32(em), avg)
    assert _rel(gy.cpu().numpy(), ry) <= TOL
    assert _rel(gg.cpu().numpy(), rg) <= TOL
    gr = gr.cpu().numpy()
    assert abs(gr[0] - re) <= 1e-8 * max(abs(re), 1e-6)
    assert abs(gr[1] - rm) <= 1e-8 * max(abs(rm), 1e-6)


def test_backward_1080p_sampled_crops():
    fr = make_config(1)
    y, g = fr["noisy"].astype(np.float32), fr["guides"].astype(np.float32)
    H, W = 1080, 1920
    G = np.random.default_rng(5).standard_normal(y.shape).astype(np.float32)
    r = 8
    gy, gg, _ = flr.denoise_backward(_t(y), _t(g), _t(G), radius=r, eps=1e-3)
    gy, gg = gy.cpu().numpy(), gg.cpu().numpy()
    m = 4 * r
    for (y0, y1, x0, x1) in [(0, 24, 0, 48), (530, 554, 950, 1000), (H - 24, H, W - 48, W)]:
        cy0, cx0 = max(y0 - m, 0), max(x0 - m, 0)
        cy1, cx1 = min(y1 + m, H), min(x1 + m, W)
        ry, rg, _, _ = flr_adjoint.flr_backward(y[:, cy0:cy1, cx0:cx1], g[:, cy0:cy1, cx0:cx1],
                                                G[:, cy0:cy1, cx0:cx1], r, _f32(1e-3))
        sl = (slice(None), slice(y0 - cy0, y1 - cy0), slice(x0 - cx0, x1 - cx0))
        assert _rel(gy[:, y0:y1, x0:x1], ry[sl]) <= TOL
        assert _rel(gg[:, y0:y1, x0:x1], rg[sl]) <= TOL


def test_backward_repeatable():
    y, g, G = _frame(dict(H=70, W=300, Q=8, C=3, config=1))
    a = flr.denoise_backward(_t(y), _t(g), _t(G))
    b = flr.denoise_backward(_t(y), _t(g), _t(G))
    for u, v in zip(a, b):
        assert torch.equal(u, v)


def test_noisy_gradient_matches_forward_kernels():
    """For fixed guides the output is linear in the noisy image, so the
    forward kernels (two-pass path) and the adjoint must satisfy
    <G, F(y + d)> - <G, F(y)> = <dL/dy, d> up to FP32 rounding."""
    y, g, G = _frame(dict(H=70, W=300, Q=8, C=3, config=1))
    d = np.random.default_rng(8).standard_normal(y.shape).astype(np.float32)
    gy, _, _ = flr.denoise_backward(_t(y), _t(g), _t(G))
    f0 = flr.denoise(_t(y), _t(g), fused="two_pass").double()
    f1 = flr.denoise(_t(y + d), _t(g), fused="two_pass").double()
    lhs = float(torch.sum(_t(G).double() * (f1 - f0)))
    rhs = float(torch.sum(gy.double() * _t(d).double()))
    assert abs(lhs - rhs) <= 1e-4 * float(torch.sum(torch.abs(gy.double() * _t(d).double())))


def test_autograd_function():
    y, g, G = _frame(dict(H=40, W=260, Q=4, C=3, seed=9))
    ty = _t(y).requires_grad_(True)
    tg = _t(g).requires_grad_(True)
    te = torch.tensor(2e-3, requires_grad=True)
    tm = torch.tensor(0.1, requires_grad=True)
    out = flr.flr(ty, tg, radius=5, eps=te, mode="paper", eps_mul=tm)
    ref_out = flr.denoise(_t(y), _t(g), radius=5, eps=2e-3, mode="paper", eps_mul=0.1,
                          fused="two_pass")
    assert torch.equal(out.detach(), ref_out)
    (out * _t(G)).sum().backward()
    gy, gg, gr = flr.denoise_backward(_t(y), _t(g), _t(G), radius=5, eps=2e-3, mode="paper",
                                      eps_mul=0.1)
    assert torch.equal(ty.grad, gy) and torch.equal(tg.grad, gg)
    ry, rg, re, rm = flr_adjoint.flr_backward(y, g, G, 5, _f32(2e-3), "paper", _f32(0.1))
    assert _rel(ty.grad.cpu().numpy(), ry) <= TOL
    assert abs(te.grad.item() - re) <= 1e-6 * abs(re)
    assert abs(tm.grad.item() - rm) <= 1e-6 * abs(rm)
