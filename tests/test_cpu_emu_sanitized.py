"""The host build of the kernels and of the library's host dispatcher
(flr_api.cpp) under AddressSanitizer and UndefinedBehaviorSanitizer.

The emulator (tests/cpu_emu) compiles the kernel sources and flr_api.cpp
with g++; here the same sources are built with -fsanitize=address,undefined
(fiber stack switches annotated for ASan) and a small case of every entry
point family runs in a subprocess with libasan preloaded. Any report
(out-of-bounds or use-after-free access, misaligned or overflowing
arithmetic, invalid shifts, ...) aborts the subprocess and fails the test;
the results must also still match the oracle.
"""
import concurrent.futures as cf

import pytest

from tests.cpu_emu.harness import run_in_subprocess

CASES = [
    dict(kind="abi_checks", H=8, W=8, Q=2, C=1, r=2),
    dict(kind="both", H=16, W=270, Q=8, C=3, r=8, tile_rows=7, frame="config", config=1),
    dict(kind="both", H=5, W=11, Q=2, C=1, r=20),
    dict(kind="stages", H=5, W=270, Q=8, C=4, r=8, tile_rows=3),
    dict(kind="raw_moments", H=5, W=270, Q=3, C=2, r=3, tile_rows=2),
    dict(kind="stages", H=6, W=100, Q=3, C=2, r=3, tile_rows=4, mode="paper", eps_mul=0.1),
    dict(kind="adjoint", H=6, W=40, Q=3, C=2, r=3),
    dict(kind="lowres", H=12, W=70, Q=3, C=2, r=0, block=4, sigma=1.0, radius_low=2),
    dict(kind="batch", H=0, W=0, Q=8, C=3, r=8, sizes=[[5, 280], [3, 30]], joint=[8, 40]),
    dict(kind="net_trace", H=5, W=9, Q=8, C=3, r=0),
    dict(kind="net_bwd", H=3, W=5, Q=8, C=3, r=0),
]


@pytest.fixture(scope="module")
def sanitized_results():
    """Every case's result (or its exception), the subprocesses run four at
    a time (each is single-process; the sanitized build happens once, under
    the harness's build lock)."""
    def one(i):
        try:
            return run_in_subprocess(CASES[i], sanitize=True, timeout=900)
        except Exception as e:  # reported by the case's own test
            return e
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        return list(ex.map(one, range(len(CASES))))


@pytest.mark.parametrize("idx", range(len(CASES)), ids=lambda i: "-".join(
    f"{k}{v}" for k, v in CASES[i].items() if k in ("kind", "H", "W", "Q", "C")))
def test_sanitized_emulated_case(idx, sanitized_results):
    spec = CASES[idx]
    res = sanitized_results[idx]
    if isinstance(res, Exception):
        raise res
    kind = spec["kind"]
    if kind == "abi_checks":
        # FLR_ERR_SHAPE x2, RADIUS x2, EPS x2, CHANNELS x3, MODE x3, SHAPE; then
        # denoise: ALIAS (out over guides), NULL, ALIGN
        assert res["codes"] == [2, 2, 3, 3, 4, 4, 5, 5, 5, 9, 9, 9, 2, 6, 1, 7], res
    elif kind == "raw_moments":
        assert res["exact"], res
    elif kind == "adjoint":
        assert res["dy_rel"] <= 1e-6 and res["dg_rel"] <= 1e-6, res
    elif kind == "lowres":
        assert res["rel"] <= 1e-6, res
    elif kind == "net_trace":
        assert res["trace_equals_forward"] and res["report"]["head_rel"] <= 2e-3, res
    elif kind == "net_bwd":
        assert max(res.values()) <= 1e-4, res
    elif kind == "batch":
        assert all(v is True or (isinstance(v, float) and v <= 1e-6) for v in res.values()), res
    else:
        for k, v in res.items():
            assert v <= 1e-4, (k, v)
