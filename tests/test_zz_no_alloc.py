"""flr_l1_loss_grad_noalloc (partial sums in the library's per-GPU scratch
array, no allocation) against flr_l1_loss_grad (the same kernels with a
caller workspace): bit for bit, on two calls in a row, the second smaller,
through the C ABI."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2410_11625_amd._lib import lib  # noqa: E402

pytestmark = pytest.mark.gpu


def _both(n, seed):
    dev = torch.device("cuda:0")
    g = torch.Generator(device="cpu").manual_seed(seed)
    out = torch.randn(n, generator=g).to(dev)
    target = torch.randn(n, generator=g).to(dev)
    target[: n // 7] = out[: n // 7]  # some exact zeros of the difference
    scale = 1.0 / n
    L = lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    need = int(L.flr_l1_workspace_bytes(n))
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    g1, l1 = torch.empty_like(out), torch.empty(1, dtype=torch.float64, device=dev)
    assert L.flr_l1_loss_grad(n, out.data_ptr(), target.data_ptr(), scale, g1.data_ptr(),
                              l1.data_ptr(), ws.data_ptr(), need, stream) == 0
    g2, l2 = torch.full_like(out, np.nan), torch.full((1,), np.nan, dtype=torch.float64,
                                                       device=dev)
    assert L.flr_l1_loss_grad_noalloc(n, out.data_ptr(), target.data_ptr(), scale,
                                      g2.data_ptr(), l2.data_ptr(), stream) == 0
    torch.cuda.synchronize()
    return g1.cpu().numpy(), l1.item(), g2.cpu().numpy(), l2.item(), out, target


def test_noalloc_equals_workspace_entry_point_twice():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    for n, seed in [(3 * 256 * 256 + 5, 1), (1234, 2)]:
        g1, l1, g2, l2, out, target = _both(n, seed)
        assert np.array_equal(g1, g2), n
        assert l1 == l2, (n, l1, l2)
        # the loss is scale (an FP32 argument) times the FP64 sum of |out - target|
        want = float(np.float32(1.0 / n)) * float(np.sum(np.abs(
            out.cpu().numpy().astype(np.float64) - target.cpu().numpy().astype(np.float64))))
        assert abs(l2 - want) <= 1e-12 * abs(want), (l2, want)


def test_noalloc_validates_before_launch():
    L = lib()
    assert L.flr_l1_loss_grad_noalloc(0, 16, 16, 1.0, 32, 48, None) == 2       # FLR_ERR_SHAPE
    assert L.flr_l1_loss_grad_noalloc(1 << 35, 16, 16, 1.0, 32, 48, None) == 2
    assert L.flr_l1_loss_grad_noalloc(8, None, 16, 1.0, 32, 48, None) == 1     # FLR_ERR_NULL
    assert L.flr_l1_loss_grad_noalloc(8, 16, 16, float("inf"), 64, 96, None) == 4
