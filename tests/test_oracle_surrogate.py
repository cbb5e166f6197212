"""Pins of the surrogate and sampler references: the FP64 MLP against
PyTorch's CPU float64 layers and autograd, its gradient against central
differences, Adam against torch.optim.Adam, BF16 rounding against torch's
bfloat16 conversion, and delayed acceptance against the analytic marginals
of a Gaussian target with a deliberately wrong surrogate. CPU only."""
import numpy as np
import pytest
import scipy.stats as ss

import pta_inputs as pi
from oracle import da, mlp

D_IN, W = 10, 32  # a narrow network keeps the checks fast; layout is generic


def torch_net(flat, d_in, width):
    import torch
    p = mlp.unpack(flat, d_in, width)
    lins = []
    for l in (1, 2, 3):
        lin = torch.nn.Linear(d_in if l == 1 else width, width, dtype=torch.float64)
        lin.weight.data = torch.tensor(p["W%d" % l])
        lin.bias.data = torch.tensor(p["b%d" % l])
        lins += [lin, torch.nn.SiLU()]
    last = torch.nn.Linear(width, 1, dtype=torch.float64)
    last.weight.data = torch.tensor(p["W4"][None, :])
    last.bias.data = torch.tensor(p["b4"])
    return torch.nn.Sequential(*lins, last)


def test_param_count_matches_architecture():
    assert mlp.n_params(10, 256) == 134657


def test_bf16_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-30, 30, 5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), ref)


def test_forward_matches_torch():
    import torch
    flat = pi.mlp_weights(D_IN, W, 1)
    flat[np.arange(flat.size) % 7 == 0] += 0.01  # nonzero biases
    x = np.random.default_rng(2).uniform(-1, 1, size=(40, D_IN))
    out, _ = mlp.forward(flat, x, D_IN, W, emulate=False)
    ref = torch_net(flat, D_IN, W)(torch.tensor(x)).detach().numpy()[:, 0]
    assert np.allclose(out, ref, rtol=1e-13, atol=1e-13)


def test_gradient_matches_autograd_and_fd():
    import torch
    flat = pi.mlp_weights(D_IN, W, 3)
    rng = np.random.default_rng(4)
    x = rng.uniform(-1, 1, size=(24, D_IN))
    t = rng.normal(size=24)
    loss, g = mlp.loss_and_grad(flat, x, t, D_IN, W, emulate=False)
    net = torch_net(flat, D_IN, W)
    lt = ((net(torch.tensor(x))[:, 0] - torch.tensor(t)) ** 2).mean()
    lt.backward()
    gp = {}
    for l, lin in zip((1, 2, 3, 4), [net[0], net[2], net[4], net[6]]):
        gp["W%d" % l] = lin.weight.grad.numpy().reshape(-1) if l == 4 else lin.weight.grad.numpy()
        gp["b%d" % l] = lin.bias.grad.numpy()
    gref = mlp.pack(gp, D_IN, W)
    assert abs(loss - lt.item()) < 1e-13
    assert np.allclose(g, gref, rtol=1e-11, atol=1e-13)
    # central differences on a few coordinates
    h = 1e-6
    for j in np.random.default_rng(5).choice(flat.size, 20, replace=False):
        fp, fm = flat.copy(), flat.copy()
        fp[j] += h
        fm[j] -= h
        lp, _ = mlp.loss_and_grad(fp, x, t, D_IN, W, emulate=False)
        lm, _ = mlp.loss_and_grad(fm, x, t, D_IN, W, emulate=False)
        assert abs((lp - lm) / (2 * h) - g[j]) <= 1e-6 * max(abs(g[j]), 1e-3)


def test_adam_matches_torch():
    import torch
    rng = np.random.default_rng(6)
    w = rng.normal(size=50)
    wt = torch.tensor(w.copy(), requires_grad=True)
    opt = torch.optim.Adam([wt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50)
    v = np.zeros(50)
    for step in range(1, 6):
        g = rng.normal(size=50)
        wt.grad = torch.tensor(g)
        opt.step()
        w, m, v = mlp.adam(w, g, m, v, step, 1e-3)
    assert np.allclose(w, wt.detach().numpy(), rtol=0, atol=1e-14)


def test_emulated_forward_is_close_to_exact():
    flat = pi.mlp_weights(D_IN, W, 7)
    x = np.random.default_rng(8).uniform(-1, 1, size=(64, D_IN))
    a, _ = mlp.forward(flat, x, D_IN, W, emulate=True)
    b, _ = mlp.forward(flat, x, D_IN, W, emulate=False)
    assert np.abs(a - b).max() < 0.05 * np.abs(b).max()
    assert not np.array_equal(a, b)


def test_emulated_gradient_matches_autograd_of_the_rounding_model():
    """The emulated backward pass places BF16 roundings where the kernels
    store BF16 values: inputs, hidden weights and activations in the forward
    pass, and the gradient with respect to each hidden pre-activation (dz,
    the MFMA operand of the backward products). Independently: PyTorch
    float64 autograd through the same forward, with torch's own bfloat16
    conversion as a straight-through rounding on the forward values and a
    rounding of the incoming gradient placed on each pre-activation. Any
    other placement (no dz rounding, rounding da instead of dz, a rounded
    output-layer gradient) fails this at the tolerance used."""
    import torch

    def rnd(x):
        return x.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    class Fwd(torch.autograd.Function):  # rounds values, passes gradients
        @staticmethod
        def forward(ctx, x):
            return rnd(x)

        @staticmethod
        def backward(ctx, g):
            return g

    class Bwd(torch.autograd.Function):  # passes values, rounds gradients
        @staticmethod
        def forward(ctx, x):
            return x.clone()

        @staticmethod
        def backward(ctx, g):
            return rnd(g)

    flat = pi.mlp_weights(D_IN, W, 11)
    flat[np.arange(flat.size) % 5 == 0] += 0.02
    rng = np.random.default_rng(12)
    B = 48
    x = rng.uniform(-1, 1, size=(B, D_IN))
    t = rng.normal(size=B)
    loss, g = mlp.loss_and_grad(flat, x, t, D_IN, W, emulate=True)
    p = {k: torch.tensor(v, requires_grad=True) for k, v in mlp.unpack(flat, D_IN, W).items()}
    a = Fwd.apply(torch.tensor(x))
    for l in (1, 2, 3):
        z = Bwd.apply(a @ Fwd.apply(p["W%d" % l]).T + p["b%d" % l])
        a = Fwd.apply(torch.nn.functional.silu(z))
    out = a @ p["W4"] + p["b4"][0]
    lt = ((out - torch.tensor(t)) ** 2).mean()
    lt.backward()
    gref = mlp.pack({k: v.grad.numpy() for k, v in p.items()}, D_IN, W)
    assert abs(loss - lt.item()) <= 1e-14 * abs(loss)
    # both sides round the same FP64 values; FP64 summation order differs
    # only at ~1e-16, which can move a value across a BF16 rounding boundary
    # in rare elements: compare with a bound far below one BF16 step
    assert np.abs(g - gref).max() <= 1e-6 * np.abs(gref).max(), np.abs(g - gref).max()


def test_affine_input_map():
    """The box map is the diagonal case of the affine map; the whitening map
    T = L^-1 (Sigma = L L^T) gives unit covariance."""
    rng = np.random.default_rng(13)
    lo, hi = rng.uniform(-5, 0, D_IN), rng.uniform(1, 6, D_IN)
    th = rng.uniform(lo, hi, size=(200, D_IN))
    T = np.diag(2.0 / (hi - lo))
    assert np.allclose(mlp.affine_inputs(th, 0.5 * (lo + hi), T),
                       mlp.standardise_inputs(th, lo, hi), rtol=0, atol=1e-14)
    A = rng.normal(size=(D_IN, D_IN))
    ens = rng.normal(size=(20000, D_IN)) @ A.T + 3.0
    L = np.linalg.cholesky(np.cov(ens, rowvar=False))
    u = mlp.affine_inputs(ens, ens.mean(0), np.linalg.inv(L))
    assert np.allclose(np.cov(u, rowvar=False), np.eye(D_IN), atol=1e-10)
    assert np.allclose(u.mean(0), 0.0, atol=1e-10)


# ------------------------------------------------------------ sampler
def test_delayed_acceptance_is_exact_with_a_wrong_surrogate():
    """2-D correlated Gaussian target; the surrogate has the wrong mean and
    width. DA marginals match the analytic ones (KS, fixed seed), as does
    plain MH; DA needs fewer exact evaluations than proposals."""
    mu = np.array([1.0, -2.0])
    C = np.array([[1.0, 0.6], [0.6, 2.0]])
    Ci = np.linalg.inv(C)
    lq = lambda x: -0.5 * (x - mu) @ Ci @ (x - mu)
    lq_bad = lambda x: -0.5 * np.sum((x - mu - 0.4) ** 2) / 1.7
    T = 60000
    rng = np.random.default_rng(9)
    eps = rng.normal(size=(T, 2)) * 1.2
    lu1, lu2 = np.log(rng.uniform(size=T)), np.log(rng.uniform(size=T))
    chain, r1, r2, n_exact = da.da_mh(lq, lq_bad, mu, T, eps, lu1, lu2)
    mh_chain, acc = da.mh(lq, mu, T, eps, lu1)
    thin = chain[2000::20]
    for k in range(2):
        p = ss.kstest(thin[:, k], ss.norm(mu[k], np.sqrt(C[k, k])).cdf).pvalue
        assert p > 1e-3, (k, p)
        p = ss.kstest(mh_chain[2000::20, k], ss.norm(mu[k], np.sqrt(C[k, k])).cdf).pvalue
        assert p > 1e-3
    assert n_exact < T and 0 < r2 <= r1 < 1
