"""Pins of the layer-by-layer network check (tests/net_check.py) on the CPU.

The check is exercised on traces made by the FP64 network oracle itself
(every activation the oracle's own BF16 rounding of the exact layer value):
such a trace must pass with no flip, and planted mistakes -- one activation
off by one BF16 unit outside a rounding band, a weight changed, the skip
halves of a concatenation swapped, a padding channel set -- must fail it.
"""
import numpy as np
import pytest

from oracle import net_ref
from synth import make_config
from synth.net_weights import make_net_weights
from tests import net_check


def _encode(x):
    """float64 BF16 values [c][h][w] -> HWC int16 bit patterns."""
    f = np.ascontiguousarray(np.moveaxis(x, 0, -1)).astype(np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def _oracle_trace(H, W, seed=2):
    fr = make_config(1, h=H, w=W)
    wts = make_net_weights(seed)
    cache = {}
    sig = net_ref.net_forward(fr["guides"], fr["noisy"], wts, cache=cache)
    acts = {}
    x0 = np.zeros((16, H, W))
    x0[:11] = cache["in3"][0]
    acts["x0"] = _encode(x0)
    for name in net_check.LAYER_IO:
        acts[name] = _encode(net_ref.bf16_round(np.maximum(cache[name][1], 0.0)))
    return fr, wts, acts, sig


@pytest.fixture(scope="module")
def trace():
    return _oracle_trace(21, 34)


def test_oracle_trace_passes_without_flips(trace):
    fr, wts, acts, sig = trace
    rep, head = net_check.check_network(acts, sig, fr["guides"], fr["noisy"], wts)
    for name, v in rep.items():
        if name != "head_rel":
            assert v[2] == 0, (name, v)
    assert rep["head_rel"] <= 1e-12
    np.testing.assert_allclose(head, sig, rtol=1e-12, atol=0)


def test_region_check_matches_whole_frame(trace):
    """A region's check reads the same device inputs the whole-frame check
    does: flips found and head values agree on the overlap."""
    fr, wts, acts, sig = trace
    _, head = net_check.check_network(acts, sig, fr["guides"], fr["noisy"], wts, (5, 17, 9, 30))
    np.testing.assert_allclose(head, sig[:, 5:17, 9:30], rtol=1e-12, atol=0)


def _copy(acts):
    return {k: v.copy() for k, v in acts.items()}


@pytest.mark.parametrize("name", ["in3", "in1", "e1b", "e2b", "d1a", "d0a", "out3"])
def test_one_ulp_outside_band_fails(trace, name):
    fr, wts, acts, sig = trace
    a = _copy(acts)
    t = a[name]
    wq = {n: (net_ref.bf16_round(w), net_ref.bf16_round(b)) for n, (w, b) in wts.items()}
    z, B = net_check.layer_exact(name, acts, wq, 0, t.shape[0], 0, t.shape[1])
    lo = net_check.bf16_relu(z - B)
    hi = net_check.bf16_relu(z + B)
    # a positive activation whose interval holds one value
    cand = np.argwhere((lo == hi) & (lo > 0))
    c, i, j = cand[len(cand) // 2]
    t[i, j, c] = np.int16(int(t[i, j, c]) + 1)  # next BF16 value up
    with pytest.raises(AssertionError):
        net_check.check_network(a, sig, fr["guides"], fr["noisy"], wts)


def test_wrong_weight_fails(trace):
    fr, wts, acts, sig = trace
    w2 = {k: (w.copy(), b.copy()) for k, (w, b) in wts.items()}
    w2["e2a"][0][3, 5, 1, 2] *= 1.5
    with pytest.raises(AssertionError):
        net_check.check_network(acts, sig, fr["guides"], fr["noisy"], w2)


def test_swapped_concatenation_fails(trace):
    """d0a reads [up2(d1), e0]; a device that concatenated [e0, up2(d1)]
    would be caught: emulate it by checking against a trace whose d0a output
    is the oracle's for the swapped input."""
    fr, wts, acts, sig = trace
    a = _copy(acts)
    wq = {n: (net_ref.bf16_round(w), net_ref.bf16_round(b)) for n, (w, b) in wts.items()}
    H, W = a["in1"].shape[:2]
    up = net_ref.upsample2(np.moveaxis(net_check.decode_bf16(a["d1b"]), -1, 0), H, W)
    e0 = np.moveaxis(net_check.decode_bf16(a["in1"]), -1, 0)
    w, b = wq["d0a"]
    z = net_ref.conv2d(np.concatenate([e0, up]), w, b)
    a["d0a"] = _encode(net_check.bf16_relu(z))
    with pytest.raises(AssertionError):
        net_check.check_network(a, sig, fr["guides"], fr["noisy"], wts)


def test_padding_and_head_mistakes_fail(trace):
    fr, wts, acts, sig = trace
    a = _copy(acts)
    a["x0"][3, 4, 13] = np.int16(0x3f80)  # 1.0 in a padding channel
    with pytest.raises(AssertionError):
        net_check.check_network(a, sig, fr["guides"], fr["noisy"], wts)
    s2 = sig.copy()
    s2[2, 7, 7] *= 1 + 1e-5  # far beyond FP32 evaluation error
    with pytest.raises(AssertionError):
        net_check.check_network(acts, s2, fr["guides"], fr["noisy"], wts)
