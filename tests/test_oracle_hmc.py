"""Pins of the oracle's HMC transition against the mathematics of the
leapfrog integrator and of the Metropolis correction: the closed-form
leapfrog map of the harmonic oscillator, time reversibility, the second
order of the energy error, and sampling of correlated and box-truncated
Gaussian targets whose moments and marginals are known. CPU only."""
import numpy as np
import pytest
import scipy.stats as ss

from oracle import hmc


def test_leapfrog_harmonic_oscillator_closed_form():
    """For l = -x^2/2 one kick-drift-kick step maps (x, p) linearly by
    [[1 - e^2/2, e], [-e (1 - e^2/4), 1 - e^2/2]]."""
    f = hmc.gaussian_target([0.0], [[1.0]])
    e, L = 0.3, 17
    x0, p0 = np.array([[0.7]]), np.array([[-1.1]])
    _, g0 = f(x0)
    x, p, _, _, _ = hmc.leapfrog(x0, p0, g0, [e], [1.0], L, f)
    M = np.array([[1 - e * e / 2, e], [-e * (1 - e * e / 4), 1 - e * e / 2]])
    ref = np.linalg.matrix_power(M, L) @ np.array([0.7, -1.1])
    assert np.allclose([x[0, 0], p[0, 0]], ref, rtol=0, atol=1e-13)


def test_leapfrog_is_reversible():
    rng = np.random.default_rng(3)
    A = rng.normal(size=(3, 3))
    f = hmc.gaussian_target([0.5, -1.0, 2.0], A @ A.T + np.eye(3))
    x0, p0 = rng.normal(size=(5, 3)), rng.normal(size=(5, 3))
    m_inv = np.array([0.5, 1.0, 2.0])
    _, g0 = f(x0)
    x, p, _, g, _ = hmc.leapfrog(x0, p0, g0, np.full(5, 0.05), m_inv, 40, f)
    xb, pb, _, _, _ = hmc.leapfrog(x, -p, g, np.full(5, 0.05), m_inv, 40, f)
    assert np.allclose(xb, x0, atol=1e-11) and np.allclose(-pb, p0, atol=1e-11)


def test_energy_error_is_second_order():
    rng = np.random.default_rng(4)
    f = hmc.gaussian_target([0.0, 0.0], [[2.0, 0.3], [0.3, 1.0]])
    x0, z = rng.normal(size=(64, 2)), rng.normal(size=(64, 2))
    l0, g0 = f(x0)
    errs = []
    for e in (0.1, 0.05, 0.025):
        L = int(round(1.0 / e))
        *_, dh = hmc.transition(x0, l0, g0, np.full(64, e), [1.0, 1.0], [-1e9] * 2, [1e9] * 2,
                                z, np.full(64, -np.inf), L, f)
        errs.append(np.sqrt(np.mean(dh ** 2)))
    r = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all((r > 3.6) & (r < 4.4)), r


def run_chains(f, x, n_iter, eps, L, m_inv, lo, hi, seed):
    rng = np.random.default_rng(seed)
    S, D = x.shape
    l, g = f(x)
    acc = 0
    for _ in range(n_iter):
        z = rng.normal(size=(S, D))
        logu = np.log(rng.random(S))
        x, l, g, a, _ = hmc.transition(x, l, g, np.full(S, eps), m_inv, lo, hi, z, logu, L, f)
        acc += a.mean()
    return x, acc / n_iter


def test_samples_correlated_gaussian():
    """4000 chains from an overdispersed start, 40 transitions with a step
    size giving ~70 % acceptance: means, covariance and marginals match."""
    mu = np.array([1.0, -2.0, 0.5])
    C = np.array([[1.0, 0.8, 0.2], [0.8, 1.0, 0.1], [0.2, 0.1, 0.25]])
    f = hmc.gaussian_target(mu, np.linalg.inv(C))
    rng = np.random.default_rng(5)
    x0 = mu + 3.0 * rng.normal(size=(4000, 3))
    x, acc = run_chains(f, x0, 40, 0.45, 6, np.ones(3), np.full(3, -1e9), np.full(3, 1e9), 6)
    assert 0.5 < acc < 0.95
    assert np.allclose(x.mean(0), mu, atol=0.06)
    assert np.allclose(np.cov(x.T), C, atol=0.06)
    for i in range(3):
        assert ss.kstest(x[:, i], "norm", args=(mu[i], np.sqrt(C[i, i]))).pvalue > 1e-3


def test_samples_box_truncated_gaussian():
    """The box prior: N(0, 1) truncated to [-0.5, 2] in the first coordinate
    (trajectories that leave the box are rejected)."""
    f = hmc.gaussian_target([0.0, 0.0], np.eye(2))
    lo, hi = np.array([-0.5, -1e9]), np.array([2.0, 1e9])
    rng = np.random.default_rng(7)
    x0 = np.column_stack([rng.uniform(-0.5, 2.0, 4000), rng.normal(size=4000)])
    x, acc = run_chains(f, x0, 40, 0.3, 5, np.ones(2), lo, hi, 8)
    assert (x[:, 0] >= -0.5).all() and (x[:, 0] <= 2.0).all()
    tn = ss.truncnorm(-0.5, 2.0)
    assert ss.kstest(x[:, 0], tn.cdf).pvalue > 1e-3
    assert ss.kstest(x[:, 1], "norm").pvalue > 1e-3


def test_accept_rule_edges():
    f = hmc.gaussian_target([0.0], [[1.0]])
    x0 = np.array([[0.0], [0.0], [0.0]])
    l0, g0 = f(x0)
    z = np.array([[1.0], [1.0], [1.0]])
    # logu = -inf always accepts inside the box; the third chain starts at the
    # box edge and leaves it
    lo, hi = np.array([-10.0]), np.array([10.0])
    x1, _, _, acc, dh = hmc.transition(x0, l0, g0, np.array([0.1, 0.1, 0.1]), [1.0], lo, hi, z,
                                       np.array([-np.inf, np.inf, -np.inf]), 3, f)
    assert acc[0] and not acc[1]
    assert np.isfinite(dh[:2]).all()
    x0e = np.array([[10.0]])
    l0e, g0e = f(x0e)
    _, _, _, acc2, dh2 = hmc.transition(x0e, l0e, np.zeros_like(g0e) + 5.0, [0.1], [1.0], lo, hi,
                                        np.array([[3.0]]), np.array([-np.inf]), 2, f)
    assert not acc2[0] and np.isinf(dh2[0])


def test_failed_density_mid_trajectory_rejects():
    """A density that fails (is not finite) at an intermediate leapfrog
    position rejects the transition even when the end point is fine, as a
    filter failure part-way along a trajectory must: 1-D standard Gaussian,
    a hole (l = -inf) around the second of four leapfrog positions. The
    same draws without the hole are accepted (log u = -inf forces accept),
    so the rejection is the hole's; a hole around the end point alone
    rejects too."""
    from oracle import hmc
    base = hmc.gaussian_target([0.0], [[1.0]])
    x0 = np.array([[-1.0]])
    l0, g0 = base(x0)
    z = np.array([[1.5]])
    eps, L = 0.4, 4
    # the positions the leapfrog visits from x0 with this momentum
    xs, x, p, g = [], x0.copy(), z.copy(), g0.copy()
    for _ in range(L):
        p = p + 0.5 * eps * g
        x = x + eps * p
        xs.append(float(x[0, 0]))
        _, g = base(x)
        p = p + 0.5 * eps * g
    assert len(set(np.round(xs, 6))) == L

    def holed(center):
        def f(xx):
            l, gg = base(xx)
            bad = np.abs(xx[:, 0] - center) < 1e-3
            return np.where(bad, -np.inf, l), gg
        return f

    args = dict(eps=np.array([eps]), m_inv=np.array([1.0]), lo=np.array([-10.0]),
                hi=np.array([10.0]), z=z, logu=np.array([-np.inf]), n_leapfrog=L)
    t, l, g, acc, dh = hmc.transition(x0, l0, g0, logl_grad=base, **args)
    assert acc[0] and t[0, 0] == xs[-1] and np.isfinite(dh[0])
    for c in (xs[1], xs[-1]):
        t, l, g, acc, dh = hmc.transition(x0, l0, g0, logl_grad=holed(c), **args)
        assert not acc[0] and t[0, 0] == x0[0, 0] and l[0] == l0[0] and dh[0] == np.inf
