"""Parity of the HIP NUTS transition (argus_nuts_step: the recursion unrolled
into a lockstep loop over leaves, one batched gradient evaluation per leaf)
with the oracle's recursive transition on the same draws (complex-step
gradients of the oracle's filter), through the C ABI.

The tree's integer outcomes (depth, leapfrog count, divergence) must be
equal: they are decided by dot products and weight comparisons whose
inputs agree to ~1e-9 relative, far from ties on these seeded cases.
Positions agree to 1e-7 of the displacement, logL to 1e-9 relative, the
acceptance statistic to 1e-7 absolute."""
import numpy as np
import pytest

import pta_inputs as pi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def argus():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2510_11077_amd as A
    return A


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build()
    return oracle


def dev(x, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype or torch.float64, device="cuda")


def compare(A, orc, d, th0, eps, inv_mass, max_depth, seed, edit=None):
    import torch
    from oracle import hmc, nuts
    S, D = th0.shape
    rng = np.random.default_rng(seed)
    z, dirs, u_top, u_sub = nuts.draws(rng, S, D, max_depth)
    if edit is not None:
        edit(z, dirs)
    lo, hi = d.lo[d.free], d.hi[d.free]
    ds = A.Dataset(d)
    t = dev(th0)
    ll, g, _ = ds.loglike_grad(t)
    i32 = torch.int32
    depth = torch.empty(S, dtype=i32, device="cuda")
    nlf = torch.empty(S, dtype=i32, device="cuda")
    div = torch.empty(S, dtype=i32, device="cuda")
    acc = torch.empty(S, dtype=torch.float64, device="cuda")
    ds.nuts_step(t, ll, g, dev(np.full(S, eps)), dev(inv_mass), dev(lo), dev(hi), dev(z),
                 dev(dirs, i32), dev(u_top), dev(u_sub), max_depth, depth, nlf, div, acc)
    f = hmc.oracle_target(d, orc)
    l0, g0 = f(th0)
    rt, rl, rg, rdepth, rn, rdiv, racc = nuts.transition(th0, l0, g0, np.full(S, eps), inv_mass,
                                                         lo, hi, z, dirs, u_top, u_sub,
                                                         max_depth, f)
    assert np.array_equal(depth.cpu().numpy(), rdepth)
    assert np.array_equal(nlf.cpu().numpy(), rn)
    assert np.array_equal(div.cpu().numpy().astype(bool), rdiv)
    gt = t.cpu().numpy()
    disp = np.max(np.abs(rt - th0), axis=1, keepdims=True)
    assert (np.abs(gt - rt) <= 1e-7 * disp).all()
    assert (np.abs(ll.cpu().numpy() - rl) <= 1e-9 * np.abs(rl)).all()
    assert (np.abs(acc.cpu().numpy() - racc) <= 1e-7).all()
    return rdepth, rn, rdiv


def test_nuts_transition_per_pulsar_model(argus, orc):
    """Starts kept 5 % of the prior width inside the box (two of this
    dataset's truths sit on the box edge): most trees reach the maximum
    depth, a few stop on a leaf that leaves the box."""
    d = pi.make_pta("t", n_psr=3, counts=[40, 25, 60], seed=7)
    width = (d.hi - d.lo)[d.free]
    lo, hi = d.lo[d.free], d.hi[d.free]
    th0 = np.clip(pi.theta_near_truth(d, 24, 25, scale=0.03), lo + 0.05 * width,
                  hi - 0.05 * width)
    depth, n, div = compare(argus, orc, d, th0, 0.05, (0.02 * width) ** 2, 5, 6)
    assert depth.max() == 5 and div.any()


def test_nuts_transition_spin_model(argus, orc):
    d = pi.make_config("cfg1")
    th0 = pi.theta_near_truth(d, 16, 26, scale=0.02)
    width = d.hi - d.lo
    depth, n, div = compare(argus, orc, d, th0, 0.3, (0.005 * width) ** 2, 6, 7)
    assert depth.max() >= 2


def test_nuts_divergence_at_the_box_edge(argus, orc):
    """Chains on the upper EFAC edge with a large outward momentum diverge in
    their first leaf (depth 0, divergent, position kept)."""
    d = pi.make_pta("t", n_psr=2, counts=[30, 20], seed=8)
    th0 = pi.theta_near_truth(d, 8, 27, scale=0.02)
    th0[:4, 2] = d.hi[2]
    width = (d.hi - d.lo)[d.free]

    def push_out(z, dirs):
        z[:4, 2] = 5.0
        dirs[:4, 0] = 1

    depth, n, div = compare(argus, orc, d, th0, 0.5, (0.02 * width) ** 2, 4, 8, push_out)
    assert div[:4].all() and (depth[:4] == 0).all()


def test_nuts_driver_carries_consistent_state(argus):
    import torch
    d = pi.make_config("cfg5")
    S = 128
    th0 = dev(pi.theta_near_truth(d, S, 28, scale=0.01))
    lo, hi = d.lo[d.free], d.hi[d.free]
    ds = argus.Dataset(d)
    h = argus.NUTS(ds, th0, lo, hi, 0.3, (0.002 * (hi - lo)) ** 2, max_depth=6, seed=3)
    for _ in range(8):
        h.step()
    torch.cuda.synchronize()
    ll, g, _ = ds.loglike_grad(h.theta)
    assert torch.equal(ll, h.logl) and torch.equal(g, h.grad)
    t = h.theta.cpu().numpy()
    assert (t >= lo).all() and (t <= hi).all()
    assert (np.abs(t - th0.cpu().numpy()).max(axis=1) > 0).mean() > 0.5
    assert int(h.depth.max().item()) >= 1
