"""GPU parity of the FLNR guide network and of FLNR denoising (Sec. 3.3).

Network (BF16 weights and activations, FP32 accumulation): every layer is
checked element by element on the BF16 inputs the device fed it, read from
a forward trace (tests/net_check.py): the device's output must equal the
oracle's BF16 rounding of the exact FP64 convolution, except where that
exact value lies within the FP32 accumulation bound of a BF16 rounding
boundary, where the neighbouring BF16 value is also accepted; the sigmoid
head must agree with the oracle's sigmoid of the exact logit to FP32
rounding and to 2e-3 relative. Comparing the final output with the oracle
network run on its own would compare where rounding flips (each one valid)
happened to occur and how later layers amplify them, not the kernels.

FLNR end to end: the device's flr_flnr_denoise against the FLR oracle run
on the guides plus the oracle's sigmoid head of the validated network, at
the BF16-path tolerance 2e-3 (the 12-guide regression with untrained guides
amplifies the FP32-level difference of the two heads, about 1e-7, to about
1.3e-4 at the worst pixel). The regression part alone is also checked on the
oracle network's output at the FP32 tolerance 1e-4, and the entry point
must equal its two parts run separately, bit for bit.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2410_11625_amd as flr  # noqa: E402
from oracle import flr_ref, net_ref  # noqa: E402
from synth import make_config  # noqa: E402
from synth.net_weights import flatten_net_weights, make_net_weights  # noqa: E402
from tests.net_check import check_network  # noqa: E402

pytestmark = pytest.mark.gpu


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
def packed(weights):
    return flr.net_pack(_t(flatten_net_weights(weights)))


def _trace(fr, packed):
    out, acts = flr.net_forward_trace(_t(fr["guides"]), _t(fr["noisy"]), packed)
    torch.cuda.synchronize()
    return out.cpu().numpy(), {k: v.cpu().numpy() for k, v in acts.items()}


def _assert_few_flips(report):
    """Flips are the rare exception (about 1e-4 of the activations where the
    FP32 sum straddles a rounding boundary); every one was already checked to
    be a valid rounding of a value within the accumulation bound."""
    for name, v in report.items():
        if name != "head_rel":
            n, band, flips = v
            assert flips <= band and flips <= max(4, n // 1000), (name, v)


@pytest.mark.parametrize("H,W", [(1, 1), (7, 3), (20, 70), (33, 131), (64, 128), (96, 250)])
def test_net_layers_valid(weights, packed, H, W):
    fr = make_config(1, h=H, w=W)
    out, acts = _trace(fr, packed)
    plain = flr.net_forward(_t(fr["guides"]), _t(fr["noisy"]), packed).cpu().numpy()
    assert np.array_equal(out, plain)  # the trace runs the forward's kernels
    report, _ = check_network(acts, out, fr["guides"], fr["noisy"], weights)
    _assert_few_flips(report)


def test_net_1080p_sampled_regions(weights, packed):
    """The full 1080p frame through the forward's kernels; every layer checked
    on sampled regions (the check needs only the device's own inputs around
    each region), including the frame's corners and ragged stride-2 edges."""
    fr = make_config(1)
    out, acts = _trace(fr, packed)
    H, W = 1080, 1920
    for region in [(0, 32, 0, 64), (520, 552, 944, 1008), (H - 32, H, W - 64, W),
                   (0, 24, W - 40, W), (700, 740, 0, 48), (333, 347, 1201, 1263)]:
        report, _ = check_network(acts, out, fr["guides"], fr["noisy"], weights, region)
        _assert_few_flips(report)


def _flnr_oracle(fr, head, region, block, r=8, eps=1e-3):
    """FLR oracle over the 8 guides and the validated network head, on
    output block (y0, y1, x0, x1); head covers `region`, which contains the
    block extended by 2r (clipped to the frame)."""
    _, H, W = fr["guides"].shape
    extra = np.full((4, H, W), np.nan)
    ry0, ry1, rx0, rx1 = region
    extra[:, ry0:ry1, rx0:rx1] = head.astype(np.float32)
    g12 = np.concatenate([fr["guides"].astype(np.float64), extra])
    return flr_ref.flr_reference_block(fr["noisy"].astype(np.float64), g12, r, eps, *block)


def _rel(got, want):
    rms = np.sqrt(np.mean(want ** 2))
    return float(np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-3 * rms)))


@pytest.mark.parametrize("H,W", [(48, 96), (64, 160)])
def test_flnr_end_to_end(weights, packed, H, W):
    fr = make_config(1, h=H, w=W)
    out, acts = _trace(fr, packed)
    report, head = check_network(acts, out, fr["guides"], fr["noisy"], weights)
    _assert_few_flips(report)
    g12 = torch.zeros((12, H, W), dtype=torch.float32, device=_dev())
    g12[:8] = _t(fr["guides"])
    got = flr.flnr_denoise(_t(fr["noisy"]), g12, packed, radius=8, eps=1e-3,
                           fused="two_pass").cpu().numpy()
    assert np.array_equal(g12[8:].cpu().numpy(), out)
    want = _flnr_oracle(fr, head, (0, H, 0, W), (0, H, 0, W))
    assert _rel(got, want) <= 2e-3, _rel(got, want)


def test_flnr_end_to_end_1080p_sampled(weights, packed):
    """FLNR at 1080p in the launch configuration the benchmark times, on
    sampled blocks: the network validated on each block's 2r neighbourhood,
    the FLR oracle on the guides plus that validated head."""
    fr = make_config(1)
    H, W = 1080, 1920
    out, acts = _trace(fr, packed)
    g12 = torch.zeros((12, H, W), dtype=torch.float32, device=_dev())
    g12[:8] = _t(fr["guides"])
    got = flr.flnr_denoise(_t(fr["noisy"]), g12, packed, radius=8, eps=1e-3,
                           fused="two_pass").cpu().numpy()
    assert np.array_equal(g12[8:].cpu().numpy(), out)
    for (y0, y1, x0, x1) in [(0, 16, 0, 32), (530, 546, 950, 982), (H - 16, H, W - 32, W)]:
        region = (max(y0 - 16, 0), min(y1 + 16, H), max(x0 - 16, 0), min(x1 + 16, W))
        report, head = check_network(acts, out, fr["guides"], fr["noisy"], weights, region)
        _assert_few_flips(report)
        want = _flnr_oracle(fr, head, region, (y0, y1, x0, x1))
        e = _rel(got[:, y0:y1, x0:x1], want)
        assert e <= 2e-3, ((y0, x0), e)


def test_net_repeatable(packed):
    fr = make_config(1, h=70, w=300)
    g, y = _t(fr["guides"]), _t(fr["noisy"])
    a = flr.net_forward(g, y, packed).cpu().numpy()
    b = flr.net_forward(g, y, packed).cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("path", ["two_pass", "fused", "stages"])
def test_flnr_regression_on_oracle_guides(weights, path):
    """FLR over 12 guides (the 8 inputs and the oracle network's 4) on the GPU
    against the FLR oracle on the same float32 guides."""
    fr = make_config(1, h=40, w=200)
    extra = net_ref.net_forward(fr["guides"], fr["noisy"], weights).astype(np.float32)
    g12 = np.concatenate([fr["guides"], extra]).astype(np.float32)
    got = flr.denoise(_t(fr["noisy"]), _t(g12), radius=8, eps=1e-3, fused=path).cpu().numpy()
    want = flr_ref.flr_reference(fr["noisy"].astype(np.float64), g12.astype(np.float64), 8, 1e-3)
    rms = np.sqrt(np.mean(want ** 2))
    rel = np.abs(got - want) / np.maximum(np.abs(want), 1e-3 * rms)
    assert rel.max() <= 1e-4, rel.max()


def test_flnr_equals_network_then_regression(packed):
    fr = make_config(1, h=64, w=300)
    H, W = 64, 300
    g12 = torch.zeros((12, H, W), dtype=torch.float32, device=_dev())
    g12[:8] = _t(fr["guides"])
    y = _t(fr["noisy"])
    out = flr.flnr_denoise(y, g12, packed, radius=8, eps=1e-3, fused="two_pass")
    extra = flr.net_forward(_t(fr["guides"]), y, packed)
    assert torch.equal(g12[8:], extra)
    ref = flr.denoise(y, g12, radius=8, eps=1e-3, fused="two_pass")
    assert torch.equal(out, ref)
    assert torch.isfinite(out).all()


def test_flnr_regression_1080p_sampled():
    """The 12-guide regression FLNR runs (flr_denoise two-pass: split moment
    walks, solve, averaging) at 1080p, in the launch configuration the
    benchmark times, on sampled blocks against the FLR oracle. The four
    extra guides are seeded smooth fields in (0, 1) standing in for the
    network's sigmoid outputs (the regression's parity does not depend on
    where its guides come from)."""
    fr = make_config(1)
    H, W = 1080, 1920
    rng = np.random.default_rng(12)
    yy, xx = np.mgrid[0:H, 0:W] / np.array([H, W])[:, None, None]
    extra = np.stack([1 / (1 + np.exp(-(np.sin(6.3 * (a * xx + b * yy) + c) * 2.0)))
                      for a, b, c in rng.uniform(0.5, 3.0, size=(4, 3))]).astype(np.float32)
    g12 = np.concatenate([fr["guides"], extra]).astype(np.float32)
    got = flr.denoise(_t(fr["noisy"]), _t(g12), radius=8, eps=1e-3,
                      fused="two_pass").cpu().numpy()
    for (y0, y1, x0, x1) in [(0, 16, 0, 32), (530, 546, 950, 982), (H - 16, H, W - 32, W)]:
        want = flr_ref.flr_reference_block(fr["noisy"].astype(np.float64),
                                           g12.astype(np.float64), 8, 1e-3, y0, y1, x0, x1)
        rms = np.sqrt(np.mean(want ** 2))
        rel = np.abs(got[:, y0:y1, x0:x1] - want) / np.maximum(np.abs(want), 1e-3 * rms)
        assert rel.max() <= 1e-4, (y0, x0, rel.max())
