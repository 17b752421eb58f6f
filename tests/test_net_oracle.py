"""Pins of the FP64 guide-network oracle (CPU only).

Each pin checks the oracle against something other than itself: explicit
loops, a different library routine, PyTorch's own BF16 conversion, exact
algebraic properties of a bias-free ReLU network, or the receptive field
implied by the architecture.
"""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import net_ref
from synth.net_weights import LAYERS, flatten_net_weights, make_net_weights


def conv_loops(x, w, b, stride):
    cout, cin, k, _ = w.shape
    _, H, W = x.shape
    p = k // 2
    Ho, Wo = (H + 2 * p - k) // stride + 1, (W + 2 * p - k) // stride + 1
    out = np.zeros((cout, Ho, Wo))
    for o in range(cout):
        for i in range(Ho):
            for j in range(Wo):
                s = float(b[o])
                for c in range(cin):
                    for u in range(k):
                        for v in range(k):
                            yy, xx = stride * i + u - p, stride * j + v - p
                            if 0 <= yy < H and 0 <= xx < W:
                                s += float(w[o, c, u, v]) * float(x[c, yy, xx])
                out[o, i, j] = s
    return out


@pytest.mark.parametrize("H,W,cin,cout,k,stride", [(5, 7, 3, 2, 3, 1), (6, 9, 2, 3, 3, 2),
                                                   (7, 5, 4, 2, 1, 1), (1, 1, 2, 2, 3, 1),
                                                   (5, 4, 1, 1, 3, 2)])
def test_conv_matches_loops(H, W, cin, cout, k, stride):
    rng = np.random.default_rng(H * 31 + W)
    x = rng.standard_normal((cin, H, W))
    w = rng.standard_normal((cout, cin, k, k))
    b = rng.standard_normal(cout)
    got = net_ref.conv2d(x, w, b, stride)
    assert got.shape == (cout, -(-H // stride), -(-W // stride))
    assert np.allclose(got, conv_loops(x, w, b, stride), rtol=0, atol=1e-12)


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((3, 12, 10))
    w = rng.standard_normal((2, 3, 3, 3))
    b = np.zeros(2)
    got = net_ref.conv2d(x, w, b, 1)
    for o in range(2):
        want = sum(correlate2d(x[c], w[o, c], mode="same", boundary="fill") for c in range(3))
        assert np.allclose(got[o], want, atol=1e-12)


def test_bf16_round_known_values():
    vals = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -7, -(1 + 2.0 ** -8 + 2.0 ** -12),
                     3.14159265, 0.0, -0.0, 2.0 ** -130])
    want = np.array([1.0, 1.0, 1 + 2.0 ** -6, 1 + 2.0 ** -7, -(1 + 2.0 ** -7), 3.140625, 0.0, 0.0,
                     2.0 ** -130])
    assert np.array_equal(net_ref.bf16_round(vals), want)


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.uniform(-30, 30, 20000),
                        rng.standard_normal(1000) * 1e-39]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(net_ref.bf16_round(x.astype(np.float64)), want)


def test_upsample_and_crop():
    x = np.arange(2 * 3 * 2, dtype=np.float64).reshape(2, 3, 2)
    u = net_ref.upsample2(x, 5, 4)
    assert u.shape == (2, 5, 4)
    for c in range(2):
        for i in range(5):
            for j in range(4):
                assert u[c, i, j] == x[c, i // 2, j // 2]


def test_layer_table_matches_parameter_shapes():
    wts = make_net_weights(2)
    assert [l[0] for l in net_ref.NET_LAYERS] == [l[0] for l in LAYERS]
    for name, cin, cout, k, _, _ in net_ref.NET_LAYERS:
        w, b = wts[name]
        assert w.shape == (cout, cin, k, k) and b.shape == (cout,)
    n = sum(cout * cin * k * k + cout for _, cin, cout, k in LAYERS)
    assert flatten_net_weights(wts).size == n


def _frame(H, W, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 1, (8, H, W)), rng.exponential(1.0, (3, H, W))


@pytest.mark.parametrize("H,W", [(16, 24), (13, 21), (1, 1), (2, 3)])
def test_output_shape_and_range(H, W):
    """Sigmoid outputs lie in (0, 1); odd sizes go through the stride-2 and
    upsampling steps."""
    g, y = _frame(H, W, H + W)
    out = net_ref.net_forward(g, y, make_net_weights(2))
    assert out.shape == (4, H, W)
    assert np.all((out > 0) & (out < 1))


def test_bias_free_network_is_positively_homogeneous():
    """Without biases the layers form a ReLU network, which satisfies
    f(2x) = 2 f(x); scaling by two also commutes with BF16 rounding, so the
    logits match exactly (input compression bypassed)."""
    g, y = _frame(20, 28, 5)
    wts = make_net_weights(2, zero_bias=True)
    z1 = net_ref.net_forward(g, y, wts, logits=True, compress=False)
    z2 = net_ref.net_forward(2 * g, 2 * y, wts, logits=True, compress=False)
    assert np.array_equal(z2, 2 * z1)


def test_receptive_field():
    """A 3x3 layer reaches one pixel of its own grid: one full-resolution
    pixel for in3, e1a, d0a, d0b and out3, two for the half-resolution layers
    (e1b, e2a, d1a, d1b) and four for e2b, plus up to 2 + 4 pixels of
    rounding through the stride-2 and upsampling steps, which bounds the reach
    of one input pixel by 5 + 8 + 4 + 6 = 23. Outputs farther away must be
    unchanged, and some nearby output must change."""
    H, W = 64, 64
    g, y = _frame(H, W, 9)
    wts = make_net_weights(2)
    base = net_ref.net_forward(g, y, wts, logits=True)
    g2 = g.copy()
    g2[:, 32, 32] += 0.5
    d = np.abs(net_ref.net_forward(g2, y, wts, logits=True) - base).max(axis=0)
    ii, jj = np.nonzero(d)
    assert ii.size > 0
    assert np.all(np.abs(ii - 32) <= 24) and np.all(np.abs(jj - 32) <= 24)


def test_skip_connections_matter():
    """Zeroing the decoder's skip half of d0a's weights changes the output
    (the concatenation order [upsampled, skip] is honoured)."""
    g, y = _frame(16, 16, 11)
    wts = make_net_weights(2)
    w, b = wts["d0a"]
    w2 = w.copy()
    w2[:, 32:] = 0
    alt = dict(wts, d0a=(w2, b))
    assert not np.array_equal(net_ref.net_forward(g, y, wts), net_ref.net_forward(g, y, alt))


# --------------------------------------------------------------------------
# Planted mistakes in the network oracle must be caught by the pins above.

def _net_battery() -> bool:
    ok = True
    rng = np.random.default_rng(21)
    for (H, W, cin, cout, k, s) in [(6, 7, 2, 2, 3, 1), (6, 9, 2, 2, 3, 2)]:
        x = rng.standard_normal((cin, H, W))
        w = rng.standard_normal((cout, cin, k, k))
        b = rng.standard_normal(cout)
        got = net_ref.conv2d(x, w, b, s)
        want = conv_loops(x, w, b, s)
        ok &= got.shape == want.shape and bool(np.allclose(got, want, atol=1e-12))
    vals = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 3.14159265])
    ok &= bool(np.array_equal(net_ref.bf16_round(vals), [1.0, 1 + 2.0 ** -6, 3.140625]))
    x = np.arange(6, dtype=np.float64).reshape(1, 3, 2)
    ok &= bool(np.array_equal(net_ref.upsample2(x, 5, 4)[0, 3], [x[0, 1, 0]] * 2 + [x[0, 1, 1]] * 2))
    return ok


def test_unmutated_net_oracle_passes_battery():
    assert _net_battery()


def _conv_flipped(x, w, b, stride=1, _orig=net_ref.conv2d):
    return _orig(x, w[:, :, ::-1, ::-1], b, stride)          # convolution instead of correlation


def _conv_no_bias(x, w, b, stride=1, _orig=net_ref.conv2d):
    return _orig(x, w, np.zeros_like(b), stride)


def _conv_odd_stride_origin(x, w, b, stride=1, _orig=net_ref.conv2d):
    return _orig(x[:, 1:, 1:] if stride == 2 else x, w, b, stride)


def _bf16_truncate(x):
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    return np.ldexp(np.trunc(np.ldexp(m, 8)), e - 8)         # truncation, not rounding


def _upsample_shifted(x, H, W):
    return x[:, np.minimum((np.arange(H) + 1) // 2, x.shape[1] - 1)][:, :, np.arange(W) // 2]


@pytest.mark.parametrize("name,fn", [("conv2d", _conv_flipped), ("conv2d", _conv_no_bias),
                                     ("conv2d", _conv_odd_stride_origin),
                                     ("bf16_round", _bf16_truncate),
                                     ("upsample2", _upsample_shifted)])
def test_planted_net_mistake_is_caught(monkeypatch, name, fn):
    monkeypatch.setattr(net_ref, name, fn)
    assert not _net_battery()


def test_input_compression():
    """Scaling the inputs changes the output (the compression is not linear),
    and the compression maps v to sign(v) log(1 + |v|) before BF16 rounding:
    an input of e - 1 reaches the first layer as exactly 1."""
    g, y = _frame(12, 12, 13)
    wts = make_net_weights(2, zero_bias=True)
    z1 = net_ref.net_forward(g, y, wts, logits=True)
    z2 = net_ref.net_forward(2 * g, 2 * y, wts, logits=True)
    assert not np.allclose(z2, 2 * z1)
    g1 = np.full_like(g, np.e - 1.0)
    y1 = np.full_like(y, np.e - 1.0)
    assert np.array_equal(net_ref.net_forward(g1, y1, wts, logits=True),
                          net_ref.net_forward(np.ones_like(g), np.ones_like(y), wts, logits=True,
                                              compress=False))
