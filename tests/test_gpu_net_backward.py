"""GPU parity of the guide network's backward (flr_net_backward).

Against the FP64 oracle oracle/net_adjoint.py (pinned to finite differences)
with the same straight-through reading of the BF16 forward: each side takes
the gradients of the exact network at its own BF16 weights and activations.

The two forwards accumulate in different precisions (FP32 on the matrix
cores, FP64 in the oracle), so an activation whose exact value lies within
the FP32 error of a BF16 rounding boundary can round to neighbouring BF16
values on the two sides; such a flip moves the next layer's values by about
one BF16 unit and so causes further flips, and the two sides differentiate
slightly different networks. Hence two tiers:

* Frames on which the forwards round alike (checked on the network output
  against the oracle: within 1e-5, which a flip exceeds): each layer's
  gradients within 1e-4 of the largest of that layer (FP32 sums over the
  frame).
* Larger frames (a ragged 37 x 70, the 256 x 256 training crop, a 1080p
  frame with grad_out on a 32 x 32 patch) with a smooth grad_out: within
  2e-2 of each layer's largest gradient, about five BF16 units (2^-8): the
  flip cascade's effect, measured at 2^-8 scale. With a random-sign grad_out
  the gradients largely cancel and the same flips weigh more, so these
  frames use a smooth one.
* accumulate=1 adds exactly; two calls are bit-identical.

For the 1080p frame only pixels within the network's reach of the patch
contribute; the oracle runs on a crop with a 64-pixel margin, aligned to 4
so that the stride-2 sampling and the upsampling phase match the full frame.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2410_11625_amd as flr  # noqa: E402
from oracle import net_adjoint, net_ref  # noqa: E402
from synth import make_config  # noqa: E402
from synth.net_weights import LAYERS, flatten_net_weights, make_net_weights  # noqa: E402

pytestmark = pytest.mark.gpu

TOL_EXACT = 1e-4
TOL_BF16 = 2e-2


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(_dev())


@pytest.fixture(scope="module")
def weights():
    return make_net_weights(2)


@pytest.fixture(scope="module")
def params(weights):
    p = _t(flatten_net_weights(weights))
    return p, flr.net_pack(p)


def _layer_errors(got, want, weights):
    out, o = {}, 0
    for name, _, _, _ in LAYERS:
        for tag, ref in (("w", want[name][0]), ("b", want[name][1])):
            n = ref.size
            g = np.asarray(got[o:o + n], np.float64).reshape(ref.shape)
            out[f"{name}.{tag}"] = float(np.max(np.abs(g - ref)) / max(np.max(np.abs(ref)), 1e-30))
            o += n
    assert o == got.size
    return out


def _oracle(guides, noisy, weights, G):
    cache = {}
    net_ref.net_forward(guides, noisy, weights, cache=cache)
    return net_adjoint.net_backward(cache, G)


def _check(got, want, weights, tol):
    assert np.all(np.isfinite(got))
    errs = _layer_errors(got, want, weights)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, bad


def _smooth(H, W, y0=0, x0=0):
    yy, xx = np.mgrid[0:H, 0:W]
    yy, xx = yy + y0, xx + x0
    return np.stack([np.cos(0.05 * xx + k) * np.sin(0.07 * yy + 2 * k) + 0.3
                     for k in range(4)]).astype(np.float32)


# (H, W, frame seed): small and ragged frames, including a single row
EXACT = [(9, 13, 1), (12, 20, 3), (16, 24, 5), (20, 33, 4), (1, 5, 1), (7, 3, 2)]


def test_net_backward_matches_oracle_where_forwards_agree(weights, params):
    p, packed = params
    checked = []
    for H, W, seed in EXACT:
        fr = make_config(1, seed=seed, h=H, w=W)
        g, y = _t(fr["guides"]), _t(fr["noisy"])
        fwd = flr.net_forward(g, y, packed).cpu().numpy()
        if np.max(np.abs(fwd - net_ref.net_forward(fr["guides"], fr["noisy"], weights))) > 1e-5:
            continue
        G = np.random.default_rng(H + W).standard_normal((4, H, W)).astype(np.float32)
        got = flr.net_backward(g, y, p, packed, _t(G)).cpu().numpy()
        _check(got, _oracle(fr["guides"], fr["noisy"], weights, G.astype(np.float64)), weights,
               TOL_EXACT)
        checked.append((H, W))
    assert len(checked) >= 4, checked


@pytest.mark.parametrize("H,W", [(37, 70), (256, 256)])
def test_net_backward_matches_oracle_bf16(weights, params, H, W):
    p, packed = params
    fr = make_config(1, seed=1, h=H, w=W)
    G = _smooth(H, W)
    got = flr.net_backward(_t(fr["guides"]), _t(fr["noisy"]), p, packed, _t(G)).cpu().numpy()
    _check(got, _oracle(fr["guides"], fr["noisy"], weights, G.astype(np.float64)), weights,
           TOL_BF16)


def test_net_backward_1080p_patch(weights, params):
    p, packed = params
    fr = make_config(1)
    H, W = fr["guides"].shape[1:]
    G = np.zeros((4, H, W), np.float32)
    y0, x0, n, m = 520, 900, 32, 64
    G[:, y0:y0 + n, x0:x0 + n] = _smooth(n, n, y0, x0)
    got = flr.net_backward(_t(fr["guides"]), _t(fr["noisy"]), p, packed, _t(G)).cpu().numpy()
    sl = (slice(None), slice(y0 - m, y0 + n + m), slice(x0 - m, x0 + n + m))
    want = _oracle(fr["guides"][sl], fr["noisy"][sl], weights, G[sl].astype(np.float64))
    _check(got, want, weights, TOL_BF16)


def test_net_backward_accumulate_and_repeat(params):
    p, packed = params
    a = make_config(1, seed=11, h=70, w=90)
    b = make_config(1, seed=12, h=70, w=90)
    Ga = _t(np.random.default_rng(1).standard_normal((4, 70, 90)))
    Gb = _t(np.random.default_rng(2).standard_normal((4, 70, 90)))
    ga = flr.net_backward(_t(a["guides"]), _t(a["noisy"]), p, packed, Ga)
    gb = flr.net_backward(_t(b["guides"]), _t(b["noisy"]), p, packed, Gb)
    acc = ga.clone()
    flr.net_backward(_t(b["guides"]), _t(b["noisy"]), p, packed, Gb, grad_params=acc,
                     accumulate=True)
    assert torch.equal(acc, ga + gb)
    assert torch.equal(gb, flr.net_backward(_t(b["guides"]), _t(b["noisy"]), p, packed, Gb))


def test_dgrad_channel_widths_bit_equal(params, monkeypatch):
    """The data gradients take 16 input channels per thread from
    FLR_DGRAD_WIDE_PX pixels up (default 2^18) and 8 below, with the same
    sum order per channel: at a threshold of one pixel (16 everywhere) the
    gradients of a small frame equal the default's bit for bit."""
    p, packed = params
    fr = make_config(1, seed=13, h=37, w=70)
    G = _t(np.random.default_rng(3).standard_normal((4, 37, 70)))
    monkeypatch.delenv("FLR_DGRAD_WIDE_PX", raising=False)
    narrow = flr.net_backward(_t(fr["guides"]), _t(fr["noisy"]), p, packed, G)
    monkeypatch.setenv("FLR_DGRAD_WIDE_PX", "1")
    wide = flr.net_backward(_t(fr["guides"]), _t(fr["noisy"]), p, packed, G)
    torch.cuda.synchronize()
    assert torch.isfinite(narrow).all()
    assert torch.equal(narrow, wide)
