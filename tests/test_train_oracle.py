"""Pins of the training-step oracle (oracle/train_ref.py), CPU only.

* AdamW against torch.optim.AdamW (the library's implementation of the same
  published method) over several steps with weight decay, in float64.
* AdamW closed forms: the first step moves every parameter by lr * g / (|g| +
  eps) (bias correction cancels the moment decay), and with zero gradient
  only the decay acts.
* The L1 gradient against central finite differences of the L1 loss.
* Planted mistakes (a missing bias correction, decay applied through the
  gradient, a sign slip) fail these pins.
"""
import numpy as np
import pytest

from oracle import train_ref


def _torch_adamw(p0, grads, lr, wd, betas=(0.9, 0.999), eps=1e-8):
    torch = pytest.importorskip("torch")
    p = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.AdamW([p], lr=lr, betas=betas, eps=eps, weight_decay=wd)
    for g in grads:
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    return p.detach().numpy()


def _oracle_adamw(p0, grads, lr, wd, fn=None):
    fn = fn or train_ref.adamw_step
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for t, g in enumerate(grads, start=1):
        p, m, v = fn(p, g, m, v, t, lr, 0.9, 0.999, 1e-8, wd)
    return p


def _case(seed=0, n=50, steps=5):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n), [rng.standard_normal(n) * (1 + k) for k in range(steps)]


def _adamw_ok(fn=None) -> bool:
    p0, grads = _case()
    want = _torch_adamw(p0, grads, 1e-2, 0.1)
    got = _oracle_adamw(p0, grads, 1e-2, 0.1, fn)
    return bool(np.allclose(got, want, rtol=1e-12, atol=1e-14))


def test_adamw_matches_library_optimizer():
    assert _adamw_ok()


def test_adamw_closed_forms():
    g = np.array([2.0, -0.5, 1e-3, 0.0])
    p0 = np.array([1.0, 1.0, -1.0, 3.0])
    p, m, v = train_ref.adamw_step(p0, g, np.zeros(4), np.zeros(4), 1, 0.1, eps=1e-8)
    assert np.allclose(p, p0 - 0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    p2, _, _ = train_ref.adamw_step(p0, np.zeros(4), np.zeros(4), np.zeros(4), 1, 0.1,
                                    weight_decay=0.5)
    assert np.allclose(p2, p0 * (1 - 0.05), rtol=1e-15)


def test_l1_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    out = rng.standard_normal(40)
    target = rng.standard_normal(40)
    scale = 1.0 / 40
    loss, grad = train_ref.l1_loss_grad(out, target, scale)
    assert loss == pytest.approx(np.mean(np.abs(out - target)), rel=1e-14)
    h = 1e-7
    for i in range(40):
        e = np.zeros(40)
        e[i] = h
        fd = (train_ref.l1_loss_grad(out + e, target, scale)[0] -
              train_ref.l1_loss_grad(out - e, target, scale)[0]) / (2 * h)
        assert fd == pytest.approx(grad[i], rel=1e-6)
    assert train_ref.l1_loss_grad(np.ones(3), np.ones(3), 1.0)[1].tolist() == [0.0, 0.0, 0.0]


def _no_bias_correction(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8,
                        weight_decay=0.0):
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    p = p * (1 - lr * weight_decay) - lr * m / (np.sqrt(v) + eps)
    return p, m, v


def _coupled_decay(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    # L2 regularisation through the gradient instead of decoupled decay
    return train_ref.adamw_step(p, np.asarray(g) + weight_decay * np.asarray(p), m, v, step, lr,
                                beta1, beta2, eps, 0.0)


def _sign_slip(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    return train_ref.adamw_step(p, -np.asarray(g), m, v, step, lr, beta1, beta2, eps,
                                weight_decay)


@pytest.mark.parametrize("fn", [_no_bias_correction, _coupled_decay, _sign_slip],
                         ids=lambda f: f.__name__)
def test_planted_optimizer_mistake_is_caught(fn):
    assert not _adamw_ok(fn)


def test_log_adam_matches_library_adam_on_the_logarithm():
    """Adam on log e against torch's Adam optimizer on a log-parameter whose
    loss gradient (by the chain rule) is e * dL/de, over several steps of
    varying gradients."""
    torch = pytest.importorskip("torch")
    e, m, v = 1e-3, 0.0, 0.0
    logp = torch.tensor([np.log(1e-3)], dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([logp], lr=0.05, betas=(0.9, 0.999), eps=1e-12)
    for t, ge in enumerate([3.0, -1.0, 2.5, 0.5, -4.0], start=1):
        e, m, v = train_ref.log_adam_step(e, ge, m, v, t, 0.05)
        opt.zero_grad()
        logp.grad = torch.tensor([float(np.exp(logp.item())) * ge], dtype=torch.float64)
        opt.step()
        assert abs(np.log(e) - logp.item()) <= 1e-12 * abs(logp.item()), t
