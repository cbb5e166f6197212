"""Pins of the oracle's NUTS transition: with one doubling it must be exactly
the Metropolis HMC transition of one leapfrog step; it must sample known
Gaussian targets (correlated, and truncated to the prior box); its
trajectories must stop near the half period of a harmonic oscillator, as
the no-U-turn criterion intends; and divergences must be flagged. CPU only."""
import numpy as np
import scipy.stats as ss

from oracle import hmc, nuts


def test_one_doubling_is_hmc_with_one_leapfrog_step():
    rng = np.random.default_rng(1)
    C = np.array([[1.0, 0.6], [0.6, 2.0]])
    f = hmc.gaussian_target([0.3, -0.2], np.linalg.inv(C))
    S = 200
    x0 = 1.5 * rng.normal(size=(S, 2))
    l0, g0 = f(x0)
    z, dirs, u_top, u_sub = nuts.draws(rng, S, 2, 1)
    dirs[:] = 1
    eps = np.full(S, 0.9)
    m_inv = np.array([1.0, 0.5])
    lo, hi = np.full(2, -1e9), np.full(2, 1e9)
    th, ll, g, depth, n, div, _ = nuts.transition(x0, l0, g0, eps, m_inv, lo, hi, z, dirs, u_top,
                                                  u_sub, 1, f)
    rt, rl, rg, acc, _ = hmc.transition(x0, l0, g0, eps, m_inv, lo, hi, z, np.log(u_top[:, 0]), 1, f)
    assert np.array_equal(th, rt) and np.array_equal(ll, rl)
    assert (n == 1).all() and 0.2 < acc.mean() < 0.98


def run(f, x, n_iter, eps, m_inv, lo, hi, max_depth, seed):
    rng = np.random.default_rng(seed)
    S, D = x.shape
    l, g = f(x)
    depths = []
    for _ in range(n_iter):
        z, dirs, u_top, u_sub = nuts.draws(rng, S, D, max_depth)
        x, l, g, depth, n, div, acc = nuts.transition(x, l, g, np.full(S, eps), m_inv, lo, hi, z,
                                                      dirs, u_top, u_sub, max_depth, f)
        depths.append(depth)
    return x, np.array(depths)


def test_samples_correlated_gaussian():
    mu = np.array([1.0, -2.0, 0.5])
    C = np.array([[1.0, 0.8, 0.2], [0.8, 1.0, 0.1], [0.2, 0.1, 0.25]])
    f = hmc.gaussian_target(mu, np.linalg.inv(C))
    rng = np.random.default_rng(5)
    x0 = mu + 2.0 * rng.normal(size=(600, 3))
    x, depths = run(f, x0, 25, 0.25, np.ones(3), np.full(3, -1e9), np.full(3, 1e9), 6, 6)
    assert np.allclose(x.mean(0), mu, atol=0.1)
    assert np.allclose(np.cov(x.T), C, atol=0.12)
    for i in range(3):
        assert ss.kstest(x[:, i], "norm", args=(mu[i], np.sqrt(C[i, i]))).pvalue > 1e-3
    assert depths[-5:].mean() > 1.5


def test_samples_box_truncated_gaussian():
    f = hmc.gaussian_target([0.0, 0.0], np.eye(2))
    lo, hi = np.array([-0.5, -1e9]), np.array([2.0, 1e9])
    rng = np.random.default_rng(7)
    x0 = np.column_stack([rng.uniform(-0.5, 2.0, 600), rng.normal(size=600)])
    x, _ = run(f, x0, 25, 0.3, np.ones(2), lo, hi, 6, 8)
    assert (x[:, 0] >= -0.5).all() and (x[:, 0] <= 2.0).all()
    assert ss.kstest(x[:, 0], ss.truncnorm(-0.5, 2.0).cdf).pvalue > 1e-3
    assert ss.kstest(x[:, 1], "norm").pvalue > 1e-3


def test_trajectory_stops_near_half_period():
    """For l = -x^2/2 (period 2 pi) the generalised criterion stops a
    trajectory once its end momenta turn against the summed momentum: no
    trajectory reaches a full period (2 pi / eps = 126 steps at eps = 0.05,
    so depth <= 7) and the median one spans between a quarter and a full
    period (31 to 126 steps); short trees come from starts near a turning
    point."""
    f = hmc.gaussian_target([0.0], [[1.0]])
    rng = np.random.default_rng(9)
    S = 200
    x0 = rng.normal(size=(S, 1))
    l0, g0 = f(x0)
    z, dirs, u_top, u_sub = nuts.draws(rng, S, 1, 10)
    _, _, _, depth, n, div, _ = nuts.transition(x0, l0, g0, np.full(S, 0.05), [1.0], [-1e9], [1e9],
                                                z, dirs, u_top, u_sub, 10, f)
    assert not div.any()
    assert np.all((depth >= 1) & (depth <= 7))
    assert np.pi / 0.1 <= np.median(n) <= 2 * np.pi / 0.05


def test_divergence_is_flagged():
    f = hmc.gaussian_target([0.0, 0.0], np.diag([1.0, 1e6]))
    rng = np.random.default_rng(10)
    x0 = rng.normal(size=(20, 2)) * [1.0, 1e-3]
    l0, g0 = f(x0)
    z, dirs, u_top, u_sub = nuts.draws(rng, 20, 2, 5)
    th, _, _, depth, n, div, _ = nuts.transition(x0, l0, g0, np.full(20, 0.5), [1.0, 1.0],
                                                 [-1e9] * 2, [1e9] * 2, z, dirs, u_top, u_sub, 5, f)
    assert div.all() and (depth == 0).all() and np.array_equal(th, x0)


def test_subtree_proposal_is_multinomial_over_its_leaves():
    """Within a subtree, the merges select each leaf with probability
    exp(-H_leaf) / sum over the subtree's leaves: 20,000 builds of one depth-3
    subtree (8 leaves, same trajectory, fresh merge uniforms) against those
    weights (chi-square). The target has a stiff direction, so the leaves'
    energies, and hence their weights, differ by up to a factor 2.4."""
    f = hmc.gaussian_target([0.0, 0.0], np.linalg.inv(np.diag([100.0, 0.05])))
    x0 = np.array([0.4, -0.3])
    p0 = np.array([5.0, 0.3])
    l0, g0 = f(x0[None, :])
    m_inv = np.array([1.0, 1.0])
    h0 = -l0[0] + 0.5 * np.sum(p0 * p0)
    lo, hi = np.full(2, -1e9), np.full(2, 1e9)
    eps = 0.4
    # the leaves and their weights, stepping the leapfrog by hand
    leaves, w = [], []
    st = (x0, p0, g0[0])
    for _ in range(8):
        t = nuts._leaf(st, 1, eps, m_inv, lo, hi, h0, f)
        leaves.append(t.prop[0])
        w.append(t.W)
        st = t.last
    w = np.exp(np.array(w) - np.max(w))
    w /= w.sum()
    assert w.max() / w.min() > 2.0
    rng = np.random.default_rng(11)
    counts = np.zeros(8)
    for _ in range(20000):
        t = nuts._build((x0, p0, g0[0]), 1, 3, eps, m_inv, lo, hi, h0, f, rng.random(7), [0])
        assert t.valid
        k = [i for i, x in enumerate(leaves) if np.array_equal(x, t.prop[0])]
        counts[k[0]] += 1
    chi2 = np.sum((counts - 20000 * w) ** 2 / (20000 * w))
    assert ss.chi2.sf(chi2, 7) > 1e-3, (counts / 20000, w)
