"""The HIP kernel sources executed on the host (tests/cpu_emu) against the oracle.

The same kernel templates and host dispatcher that make up libflr.so are
compiled with g++ against a CPU stand-in of the HIP runtime (a workgroup is
256 host threads meeting at a real barrier; every buffer ends at a guard
page; unwritten LDS reads as NaN). This checks indexing, synchronisation and
arithmetic of the kernels before and besides any GPU run. Each case runs in a
subprocess so that a crash is reported, not fatal.
"""
import concurrent.futures as cf
import json

import pytest

from tests.cpu_emu.harness import run_in_subprocess as _run_direct

_RESULTS: dict = {}


@pytest.fixture(scope="module", autouse=True)
def _run_selected_specs_concurrently(request):
    """Runs the `spec` cases of this module's selected tests four
    subprocesses at a time before the tests read their results (each case
    still runs alone in its own process; a failure is raised by its test)."""
    specs = {}
    for item in request.session.items:
        if item.module is not request.module:
            continue
        spec = getattr(getattr(item, "callspec", None), "params", {}).get("spec")
        if isinstance(spec, dict):
            specs[json.dumps(spec, sort_keys=True)] = spec

    def one(spec):
        try:
            return _run_direct(spec)
        except Exception as e:  # noqa: BLE001 - re-raised by the case's test
            return e
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        for key, res in zip(specs, ex.map(one, specs.values())):
            _RESULTS[key] = res
    yield
    _RESULTS.clear()


def run_in_subprocess(spec: dict) -> dict:
    """The case's result: run ahead of time by the module fixture, else now."""
    res = _RESULTS.get(json.dumps(spec, sort_keys=True))
    if res is None:
        return _run_direct(spec)
    if isinstance(res, Exception):
        raise res
    return res

TOL = 1e-4  # max relative error, |got - ref| / max(|ref|, 1e-3 rms(ref))

CASES = [
    # ragged and degenerate shapes
    dict(kind="both", H=9, W=11, Q=2, C=1, r=20),
    dict(kind="both", H=17, W=19, Q=2, C=3, r=0),
    dict(kind="both", H=1, W=300, Q=3, C=1, r=2),
    dict(kind="both", H=70, W=1, Q=1, C=2, r=3),
    # several strips and segments, workload-like frames
    dict(kind="both", H=30, W=500, Q=4, C=1, r=8, tile_rows=7, frame="config", config=0),
    dict(kind="both", H=41, W=260, Q=8, C=3, r=8, tile_rows=9, frame="config", config=1),
    # windows of near-constant guides: an FP32 factorisation erred by 1.9e-4 here
    dict(kind="both", H=40, W=270, Q=8, C=3, r=8, tile_rows=7, frame="config", config=1),
    # no averaging, Appendix regulariser
    dict(kind="both", H=33, W=250, Q=3, C=2, r=5, average=0, tile_rows=6),
    # 80 moment channels: the two-pass path splits the walk into two slices
    dict(kind="two_pass", H=29, W=270, Q=8, C=4, r=8, tile_rows=10),
    dict(kind="both", H=25, W=90, Q=3, C=2, r=3, mode="paper", eps_mul=0.2, offset=2.0),
]


@pytest.mark.parametrize("spec", CASES, ids=lambda s: "-".join(f"{k}{v}" for k, v in s.items()
                                                              if k in ("kind", "H", "W", "Q", "C", "r")))
def test_emulated_denoise_matches_oracle(spec):
    res = run_in_subprocess(spec)
    for k, v in res.items():
        assert v <= TOL, (k, v)


@pytest.mark.parametrize("spec", [
    dict(kind="raw_moments", H=37, W=300, Q=3, C=2, r=3, tile_rows=10),
    dict(kind="raw_moments", H=5, W=7, Q=1, C=1, r=8),
    # 80 channels: two walks over halves of the products
    dict(kind="raw_moments", H=21, W=280, Q=8, C=4, r=4, tile_rows=6),
])
def test_emulated_raw_moments_bit_exact(spec):
    res = run_in_subprocess(spec)
    assert res["exact"], res


def test_emulated_stages_match_oracle():
    res = run_in_subprocess(dict(kind="stages", H=24, W=270, Q=8, C=3, r=3, tile_rows=8,
                                 frame="config", config=1))
    assert res["moments_err"] < 1e-6
    assert res["solve_err"] < 1e-5
    assert res["apply_err"] < 1e-5


# The guide network's kernels (MFMA emulated per the 16x16x16 BF16 lane
# layout), every layer checked on the inputs the kernels fed it: the oracle's
# BF16 rounding of the exact convolution, a neighbouring value only within the
# FP32 accumulation bound of a rounding boundary (criteria: tests/net_check.py).
@pytest.mark.parametrize("H,W", [(20, 70), (33, 131), (1, 1), (7, 3)])
def test_emulated_net_layers_valid(H, W):
    res = run_in_subprocess(dict(kind="net_trace", H=H, W=W, Q=8, C=3, r=0))
    assert res["trace_equals_forward"]
    rep = res["report"]
    assert rep["head_rel"] <= 2e-3
    for name, v in rep.items():
        if name == "head_rel":
            continue
        n, band, flips = v
        assert flips <= band and flips <= max(4, n // 1000), (name, n, band, flips)


# The network's backward (flr_net_backward) against the FP64 backward oracle
# on a frame where the emulated BF16 forward rounds every activation as the
# oracle does: FP32-level agreement (criteria: tests/test_gpu_net_backward.py).
def test_emulated_net_backward_matches_oracle():
    res = run_in_subprocess(dict(kind="net_bwd", H=9, W=13, Q=8, C=3, r=0))
    assert max(res.values()) <= 1e-4, res


# The network backward's data-gradient kernel takes 16 input channels per
# thread on grids of 2^18 pixels or more and 8 below, with the same sum order
# per channel: with the threshold at one pixel (FLR_DGRAD_WIDE_PX=1, 16
# everywhere) the gradients must equal the default's bit for bit on a small
# frame.
def test_emulated_dgrad_variants_bit_equal(monkeypatch):
    spec = dict(kind="net_bwd_digest", H=9, W=13, Q=8, C=3, r=0)
    monkeypatch.delenv("FLR_DGRAD_WIDE_PX", raising=False)
    default = _run_direct(spec)  # the environment decides: never a prefetched result
    monkeypatch.setenv("FLR_DGRAD_WIDE_PX", "1")
    wide = _run_direct(spec)
    assert default["finite"] and default["sha256"] == wide["sha256"]


# The adjoint (flr_denoise_backward) against the FP64 adjoint oracle given
# the same FP32 eps and eps_mul. Its arithmetic is FP64 throughout (moments
# from FP64 window sums of anchored products, FP64 fields and sums), so the
# only difference left is the rounding of the FP32 outputs.
ADJ_TOL = 1e-6


@pytest.mark.parametrize("spec", [
    dict(kind="adjoint", H=40, W=300, Q=8, C=3, r=8, frame="config", config=1),
    dict(kind="adjoint", H=30, W=270, Q=4, C=1, r=8, frame="config", config=0),
    dict(kind="adjoint", H=21, W=40, Q=3, C=2, r=3, mode="paper", eps=1e-2, eps_mul=0.2,
         offset=2.0),
    dict(kind="adjoint", H=21, W=40, Q=3, C=2, r=3, average=0),
    dict(kind="adjoint", H=1, W=300, Q=2, C=1, r=2),
    dict(kind="adjoint", H=70, W=1, Q=1, C=2, r=3),
    dict(kind="adjoint", H=9, W=11, Q=2, C=1, r=20),
    dict(kind="adjoint", H=25, W=520, Q=8, C=4, r=12, mode="paper", eps=1e-3, eps_mul=0.05),
], ids=lambda s: "-".join(f"{k}{v}" for k, v in s.items() if k in ("H", "W", "Q", "C", "r",
                                                                    "mode", "average")))
def test_emulated_adjoint_matches_oracle(spec):
    res = run_in_subprocess(spec)
    assert res["dy_rel"] <= ADJ_TOL and res["dg_rel"] <= ADJ_TOL, res
    assert res["deps_rel"] <= 1e-9 and res["deps_mul_abs"] <= 1e-9, res


def test_emulated_adjoint_radius_zero():
    """r = 0: out = noisy, so dL/dnoisy = G exactly and nothing reaches the
    guides or the regularisers."""
    res = run_in_subprocess(dict(kind="adjoint", H=7, W=9, Q=2, C=2, r=0, absolute=1))
    assert res["dy_max"] == 0.0
    assert res["dg_max"] <= 1e-12 * res["g_max"] and res["reg_max"] <= 1e-12, res


# The paper's fast variant (flr_denoise_lowres) against its FP64 oracle with
# the same FP32 eps, eps_mul and sigma; FP64 throughout but the FP32 output.
@pytest.mark.parametrize("spec", [
    dict(kind="lowres", H=40, W=300, Q=8, C=3, r=0, frame="config", config=1),
    dict(kind="lowres", H=37, W=41, Q=3, C=2, r=0, block=4, sigma=1.0, radius_low=2,
         mode="paper", eps=1e-2, eps_mul=0.2, offset=2.0),
    dict(kind="lowres", H=1, W=300, Q=2, C=1, r=0),
    dict(kind="lowres", H=70, W=5, Q=1, C=2, r=0, block=16, sigma=0.0, radius_low=0),
    dict(kind="lowres", H=33, W=270, Q=4, C=4, r=0, block=2, sigma=2.0, radius_low=8),
    # block 1: staged interpolation over two rows; with Q=8, C=4 it does not
    # fit in LDS and one lane per pixel interpolates instead
    dict(kind="lowres", H=45, W=600, Q=4, C=2, r=0, block=1, sigma=0.7, radius_low=3),
    dict(kind="lowres", H=20, W=270, Q=8, C=4, r=0, block=1, sigma=0.7, radius_low=1),
], ids=lambda s: "-".join(f"{k}{v}" for k, v in s.items() if k in ("H", "W", "Q", "C", "block",
                                                                    "mode")))
def test_emulated_lowres_matches_oracle(spec):
    res = run_in_subprocess(spec)
    assert res["rel"] <= 1e-6, res


# Batched serving: plain frames of uneven size must equal flr_denoise
# (two-pass) frame by frame, bit for bit (same tile functions, same tiles);
# a joint frame (noisy input and guides on a grid `up` times coarser)
# against the oracle's low-resolution fit, window-averaged and bilinearly
# upsampled, with the FP32 eps the ABI carries. The persistent launch (a
# work queue over every stage's tiles, run twice) must equal one launch per
# stage bit for bit and report no failed wait; with fewer workgroups than
# compute units too (items wait on items other workgroups took).
@pytest.mark.parametrize("spec", [
    dict(kind="batch", H=0, W=0, Q=8, C=3, r=8, sizes=[[20, 280], [25, 70], [1, 260]],
         joint=[32, 300]),
    dict(kind="batch", H=0, W=0, Q=8, C=3, r=8, sizes=[[33, 270]], joint=[64, 600], up=4,
         tile_rows=7),
    dict(kind="batch", H=0, W=0, Q=8, C=3, r=8, sizes=[[40, 530], [9, 30]], joint=[24, 40],
         tile_rows=5, blocks=3),
], ids=["three-plain-one-joint", "tile7-joint-up4", "three-workgroups"])
def test_emulated_batch(spec):
    res = run_in_subprocess(spec)
    for k, v in res.items():
        if k.endswith("_equal") or k.startswith("persistent_"):
            assert v, (k, res)
    assert res["joint_rel"] <= 1e-6, res
