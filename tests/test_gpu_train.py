"""GPU tests of the FLNR training step (include/flr_train.h, FLNRTrainer).

* flr_l1_loss_grad against the oracle on the same FP32 values: the gradient
  bit for bit (scale times the sign of the same FP32 difference), the FP64
  loss within 1e-12 (summation order).
* flr_adamw_step against the FP64 AdamW oracle (pinned to the library
  optimizer) over three steps on the same FP32 gradients: FP32 arithmetic,
  so within 1e-6 of the largest parameter.
* A trainer step equals its parts (network, FLR, L1, FLR adjoint, network
  backward, AdamW) called one by one through the binding, bit for bit.
* Training works: on a fixed batch of the training workload the loss falls.
* A checkpoint (state_dict through a safetensors file) resumes the run: the
  resumed trainer's next step equals the uninterrupted one, bit for bit.
* One trainer step end to end against the oracle's loss, weight gradients
  and dL/deps, on a target placed so that every sign of out - target is
  decided with a wide margin (the L1 gradient's sign is a decision a
  rounding-level difference of the 12-guide regression could flip).
The parts' own parity is tested in test_gpu_net.py, test_gpu_adjoint.py and
test_gpu_net_backward.py.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2410_11625_amd as flr  # noqa: E402
from oracle import train_ref  # noqa: E402
from synth import make_training_batch  # noqa: E402
from synth.net_weights import flatten_net_weights, make_net_weights  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(_dev())


@pytest.mark.parametrize("n", [1, 7, 3 * 97 * 131, 3 * 256 * 256])
def test_l1_loss_grad_matches_oracle(n):
    rng = np.random.default_rng(n)
    out = rng.standard_normal(n).astype(np.float32)
    target = out.copy()
    target[::3] = rng.standard_normal(target[::3].shape).astype(np.float32)  # ties elsewhere
    scale = 1.0 / n
    g, loss = flr.l1_loss_grad(_t(out), _t(target), scale)
    want_loss, want_g = train_ref.l1_loss_grad(out, target, float(np.float32(scale)))
    assert np.array_equal(g.cpu().numpy(), want_g.astype(np.float32))
    assert abs(loss.item() - want_loss) <= 1e-12 * max(abs(want_loss), 1e-300)


def test_adamw_matches_oracle():
    n = 5003
    rng = np.random.default_rng(0)
    p0 = rng.standard_normal(n).astype(np.float32)
    p, m, v = _t(p0), _t(np.zeros(n)), _t(np.zeros(n))
    rp, rm, rv = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    lr, wd, betas, eps = 1e-2, 0.05, (0.9, 0.999), 1e-8
    f32 = lambda x: float(np.float32(x))  # noqa: E731  (the ABI carries FP32)
    for t in range(1, 4):
        g = (rng.standard_normal(n) * t).astype(np.float32)
        flr.adamw_step(p, _t(g), m, v, t, lr, betas, eps, wd)
        rp, rm, rv = train_ref.adamw_step(rp, g, rm, rv, t, f32(lr), f32(betas[0]),
                                          f32(betas[1]), f32(eps), f32(wd))
    got = p.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - rp)) <= 1e-6 * np.max(np.abs(rp))


def _crops(n=2, crop=48):
    return [{k: _t(v) for k, v in c.items()}
            for c in make_training_batch(n=n, crop=crop, frame_h=96, frame_w=128)]


def _parts(crops, p):
    """One step's losses, gradient and summed dL/d(eps), part by part."""
    packed = flr.net_pack(p)
    grad = torch.zeros_like(p)
    total = sum(c["noisy"].numel() for c in crops)
    losses, deps = [], 0.0
    for k, c in enumerate(crops):
        g12 = torch.empty((12,) + tuple(c["noisy"].shape[1:]), device=p.device)
        g12[:8].copy_(c["guides"])
        flr.net_forward(g12[:8], c["noisy"], packed, out=g12[8:])
        out = flr.denoise(c["noisy"], g12, 8, 1e-3, fused="two_pass")
        G, loss = flr.l1_loss_grad(out, c["target"], 1.0 / total)
        losses.append(loss)
        _, dg, dreg = flr.denoise_backward(c["noisy"], g12, G, 8, 1e-3)
        deps += float(dreg[0].item())
        flr.net_backward(g12[:8], c["noisy"], p, packed, dg[8:].contiguous(), grad_params=grad,
                         accumulate=k > 0)
    return torch.cat(losses), grad, deps


def test_trainer_step_equals_its_parts():
    crops = _crops()
    p0 = _t(flatten_net_weights(make_net_weights(2)))
    tr = flr.FLNRTrainer(p0.clone(), lr=1e-3, weight_decay=0.01)
    losses = tr.step(crops)
    p = p0.clone()
    want_losses, grad, _ = _parts(crops, p)
    flr.adamw_step(p, grad, torch.zeros_like(p), torch.zeros_like(p), 1, 1e-3,
                   weight_decay=0.01)
    assert torch.equal(losses, want_losses)
    assert torch.equal(tr.grad, grad)
    assert torch.equal(tr.params, p)


def test_trainer_learns_eps():
    """learn_eps: the step's dL/d(eps) is the crops' adjoint sums, and the
    device Adam step on log(eps) (its own step count) matches the oracle;
    the first step moves log eps by eps_lr against the gradient's sign."""
    crops = _crops()
    p0 = _t(flatten_net_weights(make_net_weights(2)))
    tr = flr.FLNRTrainer(p0.clone(), learn_eps=True, eps_lr=0.1)
    tr.step(crops)
    _, _, deps = _parts(crops, p0.clone())
    assert deps != 0.0
    got = float(tr.last_dreg[:, 0].sum().item())
    assert abs(got - deps) <= 1e-12 * abs(deps)
    e_ref, _, _ = train_ref.log_adam_step(float(np.float32(1e-3)), got, 0.0, 0.0, 1,
                                          float(np.float32(0.1)), float(np.float32(0.9)),
                                          float(np.float32(0.999)), float(np.float32(1e-12)))
    assert abs(tr.flr_eps - e_ref) <= 1e-6 * e_ref
    assert abs(np.log(tr.flr_eps / 1e-3) + 0.1 * np.sign(deps)) <= 1e-6
    assert float(tr.reg_state[4].item()) == 1.0


def test_reg_adam_step_matches_oracle():
    """Several device steps of Adam on (log eps, log eps_mul) against the
    oracle, with FP32 hyperparameters as the ABI carries them."""
    f32 = lambda x: float(np.float32(x))  # noqa: E731
    reg = torch.tensor([2e-3, 0.3], dtype=torch.float32, device=_dev())
    state = torch.zeros(6, dtype=torch.float64, device=_dev())
    e, em = f32(2e-3), f32(0.3)
    me = ve = mm = vm = 0.0
    rng = np.random.default_rng(4)
    for t in range(1, 6):
        dreg = rng.standard_normal((3, 2)) * [50.0, 0.2]
        flr.reg_adam_step(reg, state, torch.from_numpy(dreg).to(_dev()), 0.05, learn_mul=True)
        e, me, ve = train_ref.log_adam_step(e, float(dreg[:, 0].sum()), me, ve, t, f32(0.05),
                                            f32(0.9), f32(0.999), f32(1e-12))
        em, mm, vm = train_ref.log_adam_step(em, float(dreg[:, 1].sum()), mm, vm, t, f32(0.05),
                                             f32(0.9), f32(0.999), f32(1e-12))
        e, em = f32(e), f32(em)  # the device keeps (eps, eps_mul) in FP32
        got = reg.cpu().numpy().astype(np.float64)
        assert abs(got[0] - e) <= 1e-6 * e and abs(got[1] - em) <= 1e-6 * em, t
    assert float(state[4].item()) == 5.0


@pytest.mark.parametrize("path", ["two_pass", "fused", "stages"])
def test_regularisers_read_from_the_device(path):
    """flr_params.eps_device: the same results, bit for bit, as the same
    values passed as arguments, forward and backward."""
    fr = make_training_batch(n=1, crop=64, frame_h=96, frame_w=128)[0]
    y, g = _t(fr["noisy"]), _t(fr["guides"])
    reg = torch.tensor([3e-3, 0.2], dtype=torch.float32, device=_dev())
    for mode in ("ridge", "paper"):
        a = flr.denoise(y, g, 8, 3e-3, mode=mode, eps_mul=0.2, fused=path)
        b = flr.denoise(y, g, 8, 123.0, mode=mode, eps_mul=7.0, fused=path, eps_device=reg)
        assert torch.equal(a, b), mode
    G = _t(np.random.default_rng(1).standard_normal(fr["noisy"].shape))
    ra = flr.denoise_backward(y, g, G, 8, 3e-3, mode="paper", eps_mul=0.2)
    rb = flr.denoise_backward(y, g, G, 8, 1.0, mode="paper", eps_mul=1.0, eps_device=reg)
    for x, z in zip(ra, rb):
        assert torch.equal(x, z)


def test_training_reduces_the_loss():
    crops = _crops(n=2, crop=64)
    tr = flr.FLNRTrainer(_t(flatten_net_weights(make_net_weights(2))), lr=2e-3)
    first = tr.step(crops).sum().item()
    for _ in range(14):
        last = tr.step(crops).sum().item()
    assert np.isfinite(last) and last < first, (first, last)


@pytest.mark.parametrize("learn", [False, True])
def test_checkpoint_resume(tmp_path, learn):
    """A resumed run's next step equals the uninterrupted one bit for bit,
    with FLR's regularisers learned (Appendix mode, eps and eps_mul) too."""
    from safetensors.torch import load_file, save_file
    crops = _crops(n=2, crop=48)
    p0 = _t(flatten_net_weights(make_net_weights(2)))
    kw = dict(learn_eps=True, mode="paper", flr_eps_mul=0.1, eps_lr=0.05) if learn else {}
    a = flr.FLNRTrainer(p0.clone(), lr=1e-3, **kw)
    a.step(crops)
    a.step(crops)
    st = a.state_dict()
    f = tmp_path / "ckpt.safetensors"
    tensors = ("params", "m", "v", "reg", "reg_state")
    save_file({k: st[k] for k in tensors}, str(f))
    meta = {k: v for k, v in st.items() if k not in tensors}
    b = flr.FLNRTrainer(torch.zeros_like(p0), lr=0.5)
    b.load_state_dict({**load_file(str(f)), **meta})
    la = a.step(crops)
    lb = b.step(crops)
    assert torch.equal(la, lb) and torch.equal(a.params, b.params) and b.t == a.t == 3
    assert torch.equal(a.reg, b.reg) and torch.equal(a.reg_state, b.reg_state)
    if learn:
        assert a.flr_eps != 1e-3 and a.flr_eps_mul != 0.1


# One trainer step end to end against the oracle (oracle.net_adjoint's
# flnr_l1_gradients: the network, FLR over the 12 guides, the L1 loss, the
# FLR adjoint and the network backward, all FP64 but the network's BF16
# roundings). The L1 gradient takes the sign of out - target, a decision a
# rounding-level difference could flip; the target is therefore the
# oracle's own output moved by +-0.05 per element (seeded signs), so every
# sign is decided with a margin far above the two sides' difference. The
# frame is one on which the two network forwards round alike (checked:
# within 1e-5), so that the gradients compare at the BF16 path's 2e-3 of
# each layer's largest; dL/deps at 2e-3 relative.
def test_trainer_step_matches_oracle_gradients():
    from oracle import flr_ref, net_adjoint, net_ref
    from synth import random_frame
    from synth.net_weights import LAYERS
    dev = _dev()
    H, W, r = 20, 36, 8
    fr = random_frame(H, W, 8, 3, seed=21)
    weights = make_net_weights(3)
    eps = float(np.float32(1e-3))  # the regulariser as the device holds it
    extra = net_ref.net_forward(fr["guides"], fr["noisy"], weights, bf16=True)
    out_ref = flr_ref.flr_reference(fr["noisy"], np.concatenate([fr["guides"], extra]), r, eps)
    signs = np.where(np.random.default_rng(22).random(out_ref.shape) < 0.5, -1.0, 1.0)
    target = out_ref + 0.05 * signs
    loss, grads, deps = net_adjoint.flnr_l1_gradients(fr["guides"], fr["noisy"], target, weights,
                                                      r, eps, bf16=True)
    params = _t(flatten_net_weights(weights))
    g, y = _t(fr["guides"]), _t(fr["noisy"])
    net_out = flr.net_forward(g, y, flr.net_pack(params)).cpu().numpy()
    assert np.max(np.abs(net_out - extra)) <= 1e-5  # the forwards round alike
    tr = flr.FLNRTrainer(params.clone(), radius=r)
    losses = tr.step([dict(guides=g, noisy=y, target=_t(target))])
    torch.cuda.synchronize()
    assert abs(float(losses.sum().item()) - loss) <= 2e-3 * loss
    dreg = tr.last_dreg.cpu().numpy()
    assert abs(dreg[0, 0] - deps) <= 2e-3 * abs(deps), (dreg[0, 0], deps)
    got, o = tr.grad.cpu().numpy().astype(np.float64), 0
    for name, _, _, _ in LAYERS:
        for ref in grads[name]:
            n = ref.size
            err = np.max(np.abs(got[o:o + n].reshape(ref.shape) - ref))
            assert err <= 2e-3 * max(np.max(np.abs(ref)), 1e-30), name
            o += n
    assert o == got.size
