"""Parity of the HIP HMC transition (argus_hmc_step: leapfrog kernels around
the batched gradient sweep) with the oracle's transition (FP64 NumPy
leapfrog on the oracle's filter with complex-step gradients), given the same
momentum draws and accept uniforms, through the C ABI.

Tolerances: the two sides differ only through the gradient and logL they
evaluate (parity 1e-9 relative); over a few leapfrog steps that moves the
end point by about eps^2 m_inv L^2 1e-9 |g| and the energy error by about
1e-9 |logL|. Positions must agree to 1e-7 of the trajectory's displacement
and energy errors to 1e-6 + 1e-9 |logL|; accept decisions must be equal
wherever the oracle's margin |log u + dH| exceeds 1e-5, and rejected chains
must keep their positions bit for bit."""
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


def one_transition(A, orc, d, th0, eps, inv_mass, L, seed, edit_z=None):
    from oracle import hmc
    S, D = th0.shape
    rng = np.random.default_rng(seed)
    z = rng.normal(size=(S, D))
    if edit_z is not None:
        edit_z(z)
    logu = np.log(rng.random(S))
    lo, hi = d.lo[d.free], d.hi[d.free]
    ds = A.Dataset(d)
    t = dev(th0)
    ll, g, st = ds.loglike_grad(t)
    import torch
    acc = torch.zeros(S, dtype=torch.int32, device="cuda")
    dh = torch.empty(S, dtype=torch.float64, device="cuda")
    ds.hmc_step(t, ll, g, dev(np.full(S, eps)), dev(inv_mass), dev(lo), dev(hi), dev(z),
                dev(logu), L, acc, dh)
    f = hmc.oracle_target(d, orc)
    l0, g0 = f(th0)
    rt, rl, rg, racc, rdh = hmc.transition(th0, l0, g0, np.full(S, eps), inv_mass, lo, hi, z,
                                           logu, L, f)
    gt, gl, gacc, gdh = t.cpu().numpy(), ll.cpu().numpy(), acc.cpu().numpy(), dh.cpu().numpy()
    # accept decisions wherever the margin is clear
    margin = np.abs(logu + rdh)
    clear = ~(margin <= 1e-5)
    assert np.array_equal(gacc[clear].astype(bool), racc[clear])
    both = (gacc.astype(bool) == racc)
    # energy errors (inf for trajectories that left the box)
    fin = np.isfinite(rdh)
    assert np.array_equal(np.isfinite(gdh), fin)
    assert (np.abs(gdh[fin] - rdh[fin]) <= 1e-6 + 1e-9 * np.abs(l0[fin])).all()
    # positions: rejected chains keep theta exactly, accepted ones agree with
    # the oracle's end point relative to the displacement
    rej = both & ~racc
    assert np.array_equal(gt[rej], th0[rej])
    a = both & racc
    disp = np.max(np.abs(rt[a] - th0[a]), axis=1, keepdims=True)
    assert (np.abs(gt[a] - rt[a]) <= 1e-7 * disp + 1e-300).all()
    assert (np.abs(gl[a] - rl[a]) <= 1e-9 * np.abs(rl[a])).all()
    return gacc, racc, rdh


def test_hmc_transition_per_pulsar_model(argus, orc):
    d = pi.make_pta("t", n_psr=3, counts=[40, 25, 60], seed=7)
    S = 70
    th0 = pi.theta_near_truth(d, S, 21, scale=0.05)
    width = (d.hi - d.lo)[d.free]
    gacc, racc, rdh = one_transition(argus, orc, d, th0, 0.15, (0.02 * width) ** 2, 4, 3)
    assert 0 < racc.sum() < S or racc.all()


def test_hmc_transition_spin_model(argus, orc):
    d = pi.make_config("cfg1")
    th0 = pi.theta_near_truth(d, 64, 22, scale=0.02)
    width = d.hi - d.lo
    one_transition(argus, orc, d, th0, 0.5, (0.005 * width) ** 2, 5, 4)


def test_hmc_leaving_the_box_rejects(argus, orc):
    """Chains started on the upper edge of EFAC with a momentum draw of +5
    along it leave the box and are rejected with dH = +inf on both sides;
    the others move as the oracle's."""
    d = pi.make_pta("t", n_psr=2, counts=[30, 20], seed=8)
    S = 8
    th0 = pi.theta_near_truth(d, S, 23, scale=0.02)
    th0[:4, 2] = d.hi[2]
    width = (d.hi - d.lo)[d.free]

    def push_out(z):
        z[:4, 2] = 5.0

    gacc, racc, rdh = one_transition(argus, orc, d, th0, 0.5, (0.02 * width) ** 2, 3, 5, push_out)
    assert np.isinf(rdh[:4]).all() and not gacc[:4].any()
    assert np.isfinite(rdh[4:]).all()


def test_hmc_driver_carries_consistent_state(argus):
    """20 transitions of 256 chains on the 10-pulsar subset: the carried logL
    and gradient equal a fresh evaluation at the final positions, every
    position stays in the box, and the chains accept and move."""
    import torch
    d = pi.make_config("cfg5")
    S = 256
    th0 = dev(pi.theta_near_truth(d, S, 24, scale=0.01))
    lo, hi = d.lo[d.free], d.hi[d.free]
    ds = argus.Dataset(d)
    h = argus.HMC(ds, th0, lo, hi, 0.3, (0.002 * (hi - lo)) ** 2, 6, seed=1)
    for _ in range(20):
        h.step()
    torch.cuda.synchronize()
    ll, g, st = ds.loglike_grad(h.theta)
    assert torch.equal(ll, h.logl) and torch.equal(g, h.grad)
    t = h.theta.cpu().numpy()
    assert (t >= lo).all() and (t <= hi).all()
    assert h.acceptance() > 0.05
    assert (np.abs(t - th0.cpu().numpy()).max(axis=1) > 0).mean() > 0.5
