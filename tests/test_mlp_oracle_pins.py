"""Pins of the FP64 perceptron oracle (the warm-start network).

Each check compares the oracle with something it does not share code with:
central finite differences of its own loss (for the hand-written chain rule),
PyTorch's float64 modules, autograd and optimiser (library routines), and
identities of the Gaussian CDF.  The planted-mistake tests put plausible bugs
into the oracle on the CPU and show that these pins reject each one.
"""
import math

import numpy as np
import pytest
import torch

from oracle import mlp_oracle as mo

SMALL = (3, 5, 4, 2)
FULL = (13, 256, 256, 64)


def _params(shape, seed, scale=0.6):
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, mo.num_params(shape))


def _data(shape, batch, seed):
    rng = np.random.default_rng(seed + 1000)
    return rng.standard_normal((batch, shape[0])), rng.standard_normal((batch, shape[3]))


def _torch_net(flat, shape):
    n_in, h1, h2, n_out = shape
    net = torch.nn.Sequential(torch.nn.Linear(n_in, h1), torch.nn.GELU(approximate="none"),
                              torch.nn.Linear(h1, h2), torch.nn.GELU(approximate="none"),
                              torch.nn.Linear(h2, n_out)).double()
    W1, b1, W2, b2, W3, b3 = mo.unpack(flat, shape)
    with torch.no_grad():
        for lin, W, b in zip((net[0], net[2], net[4]), (W1, W2, W3), (b1, b2, b3)):
            lin.weight.copy_(torch.from_numpy(W))
            lin.bias.copy_(torch.from_numpy(b))
    return net


def _torch_flat_grad(net):
    return np.concatenate([p.grad.numpy().ravel() for p in net.parameters()])


# -------------------------------------------------------------- pin helpers

def fd_gradient_error(shape=SMALL, batch=7, seed=3, h=1e-6):
    """max |analytic - central difference| / max |gradient| over every parameter."""
    p = _params(shape, seed)
    x, t = _data(shape, batch, seed)
    g, _ = mo.grads(p, shape, x, t)
    fd = np.empty_like(p)
    for i in range(p.size):
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd[i] = (mo.loss(mo.forward(pp, shape, x), t) - mo.loss(mo.forward(pm, shape, x), t)) / (2 * h)
    return float(np.max(np.abs(g - fd)) / np.max(np.abs(fd)))


def torch_forward_error(shape=FULL, batch=33, seed=4):
    p = _params(shape, seed, scale=0.1)
    x, _ = _data(shape, batch, seed)
    ref = _torch_net(p, shape)(torch.from_numpy(x)).detach().numpy()
    return float(np.max(np.abs(mo.forward(p, shape, x) - ref)) / np.max(np.abs(ref)))


def torch_grad_error(shape=FULL, batch=33, seed=5):
    p = _params(shape, seed, scale=0.1)
    x, t = _data(shape, batch, seed)
    net = _torch_net(p, shape)
    out = net(torch.from_numpy(x))
    lt = torch.nn.functional.mse_loss(out, torch.from_numpy(t))
    lt.backward()
    ref = _torch_flat_grad(net)
    g, L = mo.grads(p, shape, x, t)
    return float(np.max(np.abs(g - ref)) / np.max(np.abs(ref))), abs(L - lt.item()) / lt.item()


def torch_adam_error(steps=6, seed=6, lr=1e-2):
    rng = np.random.default_rng(seed)
    n = 50
    p0 = rng.standard_normal(n)
    gs = [rng.standard_normal(n) * (10.0 ** rng.uniform(-4, 1, n)) for _ in range(steps)]
    w = torch.nn.Parameter(torch.from_numpy(p0.copy()))
    opt = torch.optim.Adam([w], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(n), np.zeros(n)
    err = 0.0
    for k, g in enumerate(gs, start=1):
        w.grad = torch.from_numpy(g.copy())
        opt.step()
        p, m, v = mo.adam_step(p, g, m, v, k, lr)
        err = max(err, float(np.max(np.abs(p - w.detach().numpy()))))
    return err


# ------------------------------------------------------------------- pins

def test_gelu_matches_torch_exact_gelu():
    z = np.linspace(-9, 9, 4001)
    ref = torch.nn.functional.gelu(torch.from_numpy(z), approximate="none").numpy()
    np.testing.assert_allclose(mo.gelu(z), ref, rtol=1e-12, atol=1e-15)


def test_gelu_identities():
    """Phi(-z) = 1 - Phi(z) gives gelu(-z) = gelu(z) - z; gelu(0) = 0,
    gelu'(0) = 1/2; gelu(z) -> z and gelu'(z) -> 1 for large z."""
    z = np.linspace(-6, 6, 241)
    np.testing.assert_allclose(mo.gelu(-z), mo.gelu(z) - z, atol=1e-14)
    assert mo.gelu(0.0) == 0.0 and mo.gelu_prime(0.0) == 0.5
    assert mo.gelu(12.0) == 12.0 and mo.gelu_prime(12.0) == 1.0
    assert abs(mo.gelu(-12.0)) < 1e-30


def test_gelu_prime_matches_autograd_and_differences():
    z = np.linspace(-7, 7, 1001)
    zt = torch.from_numpy(z).requires_grad_(True)
    torch.nn.functional.gelu(zt, approximate="none").sum().backward()
    np.testing.assert_allclose(mo.gelu_prime(z), zt.grad.numpy(), rtol=1e-13, atol=1e-15)
    h = 1e-5
    fd = (mo.gelu(z + h) - mo.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(mo.gelu_prime(z), fd, atol=1e-9)


def test_forward_matches_torch_modules():
    assert torch_forward_error() < 1e-13


def test_loss_is_mean_squared_error():
    o = np.array([[1.0, 2.0], [3.0, 4.0], [5.0, 6.0]])
    t = np.array([[1.0, 0.0], [0.0, 4.0], [5.0, 7.0]])
    assert mo.loss(o, t) == (4.0 + 9.0 + 1.0) / 6.0
    assert mo.loss(o, o) == 0.0


def test_gradient_matches_central_differences():
    assert fd_gradient_error() < 1e-7


def test_gradient_matches_torch_autograd_full_width():
    eg, el = torch_grad_error()
    assert eg < 1e-12 and el < 1e-13


def test_gradient_is_zero_at_a_perfect_fit():
    p = _params(SMALL, 9)
    x, _ = _data(SMALL, 5, 9)
    g, L = mo.grads(p, SMALL, x, mo.forward(p, SMALL, x))
    assert L == 0.0 and not np.any(g)


def test_adam_matches_torch_optimizer():
    assert torch_adam_error() < 1e-14


def test_adam_first_step_moves_each_parameter_by_lr():
    """Bias correction makes the first step lr * g / (|g| + eps)."""
    g = np.array([3.0, -0.25, 1e-3, 0.0])
    p, _, _ = mo.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.1)
    np.testing.assert_allclose(p, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_layout_counts():
    assert mo.num_params(FULL) == 13 * 256 + 256 + 256 * 256 + 256 + 64 * 256 + 64 == 85824
    W1, b1, W2, b2, W3, b3 = mo.unpack(np.arange(mo.num_params(SMALL), dtype=float), SMALL)
    assert W1.shape == (5, 3) and b1[0] == 15 and W2.shape == (4, 5) and W3.shape == (2, 4) and b3[-1] == 53


# ----------------------------------------------------- planted mistakes

@pytest.mark.parametrize("mutant", ["gelu_tanh", "drop_pdf_term", "transposed_dw", "no_bias_correction",
                                    "loss_not_mean"])
def test_pins_catch_planted_mistakes(mutant, monkeypatch):
    if mutant == "gelu_tanh":
        monkeypatch.setattr(mo, "gelu", lambda z: 0.5 * np.asarray(z) * (1 + np.tanh(
            math.sqrt(2 / math.pi) * (np.asarray(z) + 0.044715 * np.asarray(z) ** 3))))
        assert torch_forward_error() > 1e-6
    elif mutant == "drop_pdf_term":
        monkeypatch.setattr(mo, "gelu_prime", lambda z: 0.5 * (1 + mo.erf(np.asarray(z) / math.sqrt(2))))
        assert fd_gradient_error() > 1e-3
    elif mutant == "transposed_dw":
        orig = mo.grads

        def bad(flat, shape, x, t):
            g, L = orig(flat, shape, x, t)
            n_in, h1 = shape[0], shape[1]
            g = g.copy()
            g[: h1 * n_in] = g[: h1 * n_in].reshape(h1, n_in).T.ravel()
            return g, L
        monkeypatch.setattr(mo, "grads", bad)
        assert fd_gradient_error() > 1e-3
    elif mutant == "no_bias_correction":
        def bad(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
            m = beta1 * m + (1 - beta1) * g
            v = beta2 * v + (1 - beta2) * g * g
            return p - lr * m / (np.sqrt(v) + eps), m, v
        monkeypatch.setattr(mo, "adam_step", bad)
        assert torch_adam_error() > 1e-4
    else:
        monkeypatch.setattr(mo, "loss", lambda o, t: float(np.sum((np.asarray(o) - np.asarray(t)) ** 2)))
        assert fd_gradient_error() > 1e-3


# ------------------------------------------------ initial parameters, output scaling

def test_splitmix64_published_values():
    """The SplitMix64 stream started at 0 begins 0xE220A8397B1DCDAF,
    0x6E789E6AA1B965F4, 0x06C45D188009454F (the generator's widely published
    reference outputs)."""
    v = [int(x) for x in mo.splitmix64(0, [0, 1, 2])]
    assert v == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_init_params_bounds_and_moments():
    shape = (13, 256, 256, 64)
    p = mo.init_params(shape, 5)
    assert p.shape == (mo.num_params(shape),)
    W1, b1, W2, b2, W3, b3 = mo.unpack(p, shape)
    for w, fan in ((W1, 13), (b1, 13), (W2, 256), (b2, 256), (W3, 256), (b3, 256)):
        bound = 1.0 / math.sqrt(fan)
        assert np.all(np.abs(w) <= bound)
    # uniform on [-b, b): mean 0, variance b^2 / 3
    w = W2.ravel() * 16.0
    assert abs(w.mean()) < 0.01 and abs(w.var() - 1.0 / 3.0) < 0.01
    assert not np.array_equal(p, mo.init_params(shape, 6))


def test_output_scaling_matches_torch():
    rng = np.random.default_rng(3)
    T = rng.standard_normal((500, 7)) * rng.uniform(0.1, 5, 7) + rng.uniform(-3, 3, 7)
    mu, sd = mo.output_scaling(T)
    tt = torch.from_numpy(T)
    np.testing.assert_allclose(mu, tt.mean(0).numpy(), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(sd, tt.std(0).numpy(), rtol=1e-12)


def test_scaled_forward_equals_folded_network():
    """sd * (W3 h + b3) + mu is the network whose last layer is
    (diag(sd) W3, sd b3 + mu)."""
    shape = (5, 12, 9, 4)
    rng = np.random.default_rng(8)
    p = rng.standard_normal(mo.num_params(shape)) * 0.3
    mu, sd = rng.standard_normal(4), rng.uniform(0.5, 3, 4)
    q = p.copy()
    n_out, h2 = 4, 9
    w3 = len(q) - n_out - n_out * h2
    q[w3: w3 + n_out * h2] = (q[w3: w3 + n_out * h2].reshape(n_out, h2) * sd[:, None]).ravel()
    q[-n_out:] = q[-n_out:] * sd + mu
    x = rng.standard_normal((6, 5))
    np.testing.assert_allclose(mo.forward_scaled(p, shape, x, mu, sd), mo.forward(q, shape, x), rtol=1e-12, atol=1e-12)


def test_scaled_gradient_finite_differences():
    shape = (4, 6, 5, 3)
    rng = np.random.default_rng(9)
    p = rng.standard_normal(mo.num_params(shape)) * 0.4
    x = rng.standard_normal((7, 4))
    t = rng.standard_normal((7, 3)) * 2 + 1
    mu, sd = mo.output_scaling(t)
    g, L = mo.grads_scaled(p, shape, x, t, mu, sd)

    def lossf(q):
        return mo.loss(mo.forward(q, shape, x), (t - mu) / sd)

    assert L == pytest.approx(lossf(p), rel=1e-14)
    h = 1e-6
    for k in rng.choice(len(p), 12, replace=False):
        e = np.zeros_like(p)
        e[k] = h
        fd = (lossf(p + e) - lossf(p - e)) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-9)
