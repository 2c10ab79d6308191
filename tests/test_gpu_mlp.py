"""GPU parity of the warm-start perceptron kernels against the FP64 oracle,
per-system stop tolerances of the batched form, and the gain of the learned
warm start on held-out systems of the radial-basis family."""
import numpy as np
import pytest

import oracle
from oracle import mlp_oracle as mo
from workloads import gen

pytestmark = pytest.mark.gpu

FULL = (13, 256, 256, 64)
ODD = (3, 70, 130, 5)


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def blocks(flat, shape):
    return dict(zip(["W1", "b1", "W2", "b2", "W3", "b3"], mo.unpack(np.asarray(flat, np.float64), shape)))


def setup(lib, shape, batch, seed):
    rng = np.random.default_rng(seed)
    p = rng.uniform(-0.15, 0.15, mo.num_params(shape)).astype(np.float32)
    x = rng.standard_normal((batch, shape[0])).astype(np.float32)
    t = rng.standard_normal((batch, shape[3])).astype(np.float32)
    net = lib.MLP(*shape)
    assert net.num_params == mo.num_params(shape)
    net.set_params(dev(p))
    return net, p, x, t


@pytest.mark.parametrize("shape,batch", [(FULL, 300), (FULL, 1), (ODD, 65), (FULL, 4096)])
def test_forward_matches_oracle(lib, shape, batch):
    say("mlp forward", shape, batch)
    net, p, x, _ = setup(lib, shape, batch, 1)
    got = net.forward(dev(x)).cpu().numpy()
    ref = mo.forward(p.astype(np.float64), shape, x.astype(np.float64))
    assert rel(got, ref) <= 1e-5
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref))
    assert np.array_equal(net.get_params().cpu().numpy(), p)


@pytest.mark.parametrize("shape,batch", [(FULL, 256), (ODD, 65), (FULL, 1000)])
def test_gradients_match_oracle(lib, shape, batch):
    say("mlp grads", shape, batch)
    net, p, x, t = setup(lib, shape, batch, 2)
    g, L = net.grads(dev(x), dev(t))
    gref, Lref = mo.grads(p.astype(np.float64), shape, x.astype(np.float64), t.astype(np.float64))
    assert L == pytest.approx(Lref, rel=1e-5)
    got, ref = blocks(g.cpu().numpy(), shape), blocks(gref, shape)
    for k in got:
        assert rel(got[k], ref[k]) <= 1e-5, k


def test_adam_steps_match_oracle(lib):
    """Three training steps; each is checked against the oracle's Adam fed
    with the gradient the kernels computed at the same parameters."""
    shape, batch, lr = FULL, 256, 1e-3
    net, p, x, t = setup(lib, shape, batch, 3)
    xd, td = dev(x), dev(t)
    pr, m, v = p.astype(np.float64), np.zeros(p.size), np.zeros(p.size)
    for k in range(1, 4):
        g, _ = net.grads(xd, td)
        before = net.get_params().cpu().numpy().astype(np.float64)
        L = net.train_step(xd, td, lr, want_loss=True)
        after = net.get_params().cpu().numpy().astype(np.float64)
        pr, m, v = mo.adam_step(before, g.cpu().numpy().astype(np.float64), m, v, k, lr)
        assert np.all(np.abs(after - pr) <= 4 * 2.0 ** -24 * np.abs(pr) + 1e-4 * lr), k
        assert np.isfinite(L)
    # the parameters moved by about lr per step
    assert 0.5 * lr < np.mean(np.abs(after - p)) / 3 <= lr * 1.0001


def test_set_params_resets_adam(lib):
    shape, batch = ODD, 32
    net, p, x, t = setup(lib, shape, batch, 4)
    net.train_step(dev(x), dev(t), 1e-2)
    one = net.get_params().cpu().numpy()
    net.set_params(dev(p))
    net.train_step(dev(x), dev(t), 1e-2)
    assert np.array_equal(net.get_params().cpu().numpy(), one)


@pytest.mark.parametrize("shape,seed", [(FULL, 0), (ODD, 12345), (FULL, 2 ** 63 + 7)])
def test_initial_parameters_match_oracle(lib, shape, seed):
    """The library draws the initial parameters itself (SplitMix64 stream,
    uniform in +-1/sqrt(fan_in)): bitwise the oracle's draw."""
    net = lib.MLP(*shape, seed=seed)
    got = net.get_params().cpu().numpy()
    ref = mo.init_params(shape, seed).astype(np.float32)
    assert np.array_equal(got, ref)


def test_output_scaling_matches_oracle(lib):
    """Targets standardised per output by the library: the fitted mean and
    sample standard deviation, the forward pass in target units, and the
    gradient of the loss on standardised targets, against the oracle."""
    shape, batch = FULL, 300
    net, p, x, _ = setup(lib, shape, batch, 5)
    rng = np.random.default_rng(6)
    T = (rng.standard_normal((batch, shape[3])) * rng.uniform(0.01, 30, shape[3])
         + rng.uniform(-50, 50, shape[3])).astype(np.float32)
    net.fit_output_scaling(dev(T))
    musd = net.output_scaling().cpu().numpy().astype(np.float64)
    mu, sd = mo.output_scaling(T.astype(np.float64))
    np.testing.assert_allclose(musd[:64], mu.astype(np.float32), rtol=2 ** -23, atol=1e-30)
    np.testing.assert_allclose(musd[64:], sd.astype(np.float32), rtol=2 ** -23)
    mu32, sd32 = musd[:64], musd[64:]
    got = net.forward(dev(x)).cpu().numpy()
    ref = mo.forward_scaled(p.astype(np.float64), shape, x.astype(np.float64), mu32, sd32)
    assert rel(got, ref) <= 1e-5
    g, L = net.grads(dev(x), dev(T))
    gref, Lref = mo.grads_scaled(p.astype(np.float64), shape, x.astype(np.float64), T.astype(np.float64), mu32, sd32)
    assert L == pytest.approx(Lref, rel=1e-5)
    got, refb = blocks(g.cpu().numpy(), shape), blocks(gref, shape)
    for k in got:
        assert rel(got[k], refb[k]) <= 1e-5, k


def test_batched_per_system_tolerance(lib):
    b = gen.batch(seed=12, count=20, m_lo=256, m_hi=4096, n_lo=8, n_hi=64)
    tols = np.where(np.arange(b.count) % 2 == 0, 1e-3, 0.0)
    say("batched per-system tol")
    r = lib.solve_batched(dev(b.Xpool), dev(b.ypool), b.table, max_sweeps=300, stop=lib.STOP_REL_RESID,
                          tol=0.05, tols=tols)
    refs = oracle.solve_batch(b, max_sweeps=300, stop=oracle.STOP_REL_RESID, tol=0.05, tols=tols)
    agree = sum(int(r.sweeps[i] == refs[i].sweeps) for i in range(b.count))
    assert agree >= b.count - 2
    assert any(refs[i].sweeps != refs[i + 1].sweeps for i in range(0, b.count, 2))


def test_learned_warm_start_gains(lib):
    """Train the network on solver labels of a small radial-basis family
    (m = 512, n = 32, K = 40 sweeps) and check that, on held-out systems,
    starting from its prediction reaches each system's K-sweep residual in
    fewer sweeps than starting from zero."""
    from paper_2104_12570_amd import warmstart
    from workloads.rbf_torch import rbf_pool
    import torch
    m, n, K = 512, 32, 40
    Ptr, Ttr = gen.rbf_params(21, 4096, m=m)
    Pte, Tte = gen.rbf_params(22, 256, m=m)
    say("warm start: labels")
    Xtr, ytr, tabtr = rbf_pool(Ptr, Ttr, n=n, device="cuda")
    lab = warmstart.label(Xtr, ytr, tabtr, K)
    ws = warmstart.WarmStart(13, n, seed=0)
    say("warm start: training")
    hist = ws.fit(dev(gen.rbf_features(Ptr)), lab.a, epochs=200, batch=256, lr=2e-3, seed=0)
    assert hist[-1] < 0.5 * hist[0]
    Xte, yte, tabte = rbf_pool(Pte, Tte, n=n, device="cuda")
    ref = warmstart.label(Xte, yte, tabte, K)
    a0 = ws.predict(dev(gen.rbf_features(Pte)))
    say("warm start: held-out solves")
    warm = warmstart.solve_from(Xte, yte, tabte, a0, tols=ref.tau, max_sweeps=K)
    zero = warmstart.solve_from(Xte, yte, tabte, None, tols=ref.tau * (1 + 1e-6), max_sweeps=K)
    say("sweeps zero", zero.sweeps.mean(), "warm", warm.sweeps.mean(), "fallback", len(warm.fallback))
    assert zero.sweeps.mean() >= K - 0.5
    # the systems the prediction brought to their target needed far fewer
    # sweeps; the others were solved again from zero (the fallback), whose
    # answer is then the zero-start one
    reached = np.setdiff1d(np.arange(len(ref.tau)), warm.fallback)
    assert len(reached) >= 0.5 * len(ref.tau), len(reached)
    assert warm.sweeps[reached].mean() < 0.8 * K, warm.sweeps[reached].mean()
    if len(warm.fallback):
        np.testing.assert_allclose(warm.final_rel_resid[warm.fallback], zero.final_rel_resid[warm.fallback],
                                   rtol=1e-6)
    # the warm start is a starting point only: its answers are judged by the same FP64 check
    assert np.all(np.isfinite(warm.final_rel_resid))
    assert np.median(warm.final_rel_resid / np.maximum(ref.tau, 1e-30)) <= 1.01


def test_warm_start_full_size_sampled(lib):
    """The held-out set at full size (2000 systems, m = 4096, n = 64) in the
    configuration the benchmark times (network forward into the a0 pool of a
    recorded batched solve with per-system tolerances): sampled rows of a0
    against the oracle's forward with the trained parameters, and sampled
    solves against the oracle run from the same a0 for the same sweeps."""
    from paper_2104_12570_amd import warmstart
    from workloads.rbf_torch import rbf_pool
    import torch
    K = 100
    Ptr, Ttr = gen.rbf_params(5, 2048)
    Pte, Tte = gen.rbf_params(6, 2000)
    say("warm start full size: labels")
    Xtr, ytr, tabtr = rbf_pool(Ptr, Ttr, device="cuda")
    lab = warmstart.label(Xtr, ytr, tabtr, K)
    ws = warmstart.WarmStart(13, 64, seed=0)
    ws.fit(dev(gen.rbf_features(Ptr)), lab.a, epochs=10, batch=512, lr=2e-3)
    del Xtr, ytr
    Xte, yte, tabte = rbf_pool(Pte, Tte, device="cuda")
    ref = warmstart.label(Xte, yte, tabte, K)
    feats = gen.rbf_features(Pte)
    a0 = torch.empty(2000 * 64, dtype=torch.float32, device="cuda")
    plan = lib.BatchPlan(Xte, yte, tabte, a0pool=a0, max_sweeps=K, stop=lib.STOP_REL_RESID, tols=ref.tau)
    say("warm start full size: solve")
    ws.predict(dev(feats), out=a0)
    plan.launch()
    r = plan.results()
    params = ws.params().cpu().numpy().astype(np.float64)
    musd = ws.net.output_scaling().cpu().numpy().astype(np.float64)
    a0h = a0.view(2000, 64).cpu().numpy()
    a = r.a.cpu().numpy()
    Xh, yh = Xte.cpu().numpy(), yte.cpu().numpy()
    rng = np.random.default_rng(1)
    for i in rng.choice(2000, 10, replace=False):
        fwd = mo.forward_scaled(params, FULL, feats[i: i + 1].astype(np.float64), musd[:64], musd[64:])[0]
        assert rel(a0h[i], fwd) <= 1e-5, i
        Xt = Xh[i * 64 * 4096: (i + 1) * 64 * 4096].reshape(64, 4096)
        y = yh[i * 4096: (i + 1) * 4096]
        o = oracle.solve(Xt, y, 4096, a0=a0h[i].astype(np.float64), max_sweeps=int(r.sweeps[i]))
        say(i, r.sweeps[i], rel(a[i * 64: (i + 1) * 64], o.a), r.final_rel_resid[i],
            oracle.final_rel_resid(Xt, y, 4096, o.a))
        assert rel(a[i * 64: (i + 1) * 64], o.a) <= 1e-5, i
        assert r.final_rel_resid[i] == pytest.approx(oracle.final_rel_resid(Xt, y, 4096, o.a), rel=1e-4)
