"""Hamiltonian Monte Carlo transition (FP64 reference), the gradient-based
sampler the likelihood and its gradient feed (paper: Functionality,
"Sampler Integration"). Textbook HMC (Duane et al. 1987; Neal 2011): for a
chain at theta with log-density l(theta) and gradient g,

    p = z / sqrt(m_inv)                       (momentum ~ N(0, M), M = 1/m_inv)
    H0 = -l(theta) + 1/2 sum(m_inv p^2)
    L leapfrog steps of size eps:
        p <- p + eps/2 g;  theta <- theta + eps m_inv p;  g <- grad l(theta);
        p <- p + eps/2 g
    H1 = -l(theta') + 1/2 sum(m_inv p'^2)
    accept when log u < H0 - H1 (a NaN H1 rejects)

with a uniform prior on the box [lo, hi]: a trajectory that leaves the box,
or whose density fails, at any leapfrog position is rejected. z (standard normal
draws) and log u are inputs, so a transition is a deterministic function of
them.

TEST INFRASTRUCTURE ONLY: imported by tests, never by the product path.
"""
from __future__ import annotations

import numpy as np


def leapfrog(x, p, g, eps, m_inv, n_leapfrog, logl_grad, lo=None, hi=None):
    """n_leapfrog kick-drift-kick steps from (x, p) with g = grad l(x):
    returns (x, p, l(x), g, inside) at the end; inside is False for chains
    whose position left [lo, hi] or whose density failed (l not finite) at
    any step."""
    eps = np.asarray(eps, np.float64).reshape(-1, 1)
    m_inv = np.asarray(m_inv, np.float64).reshape(1, -1)
    x = np.asarray(x, np.float64).copy()
    p = np.asarray(p, np.float64).copy()
    g = np.asarray(g, np.float64).copy()
    inside = np.ones(x.shape[0], bool)
    l1 = None
    for _ in range(n_leapfrog):
        p = p + 0.5 * eps * g
        x = x + eps * m_inv * p
        if lo is not None:
            inside &= np.all((x >= lo) & (x <= hi), axis=1)
        l1, g = logl_grad(x)
        inside &= np.isfinite(l1)
        p = p + 0.5 * eps * g
    return x, p, l1, g, inside


def transition(theta, logl, grad, eps, m_inv, lo, hi, z, logu, n_leapfrog, logl_grad):
    """One HMC transition for S chains.

    theta [S, D], logl [S], grad [S, D]: the current state and l, grad l at it;
    eps [S]; m_inv, lo, hi [D]; z [S, D]; logu [S]; logl_grad(theta [S, D])
    -> (l [S], g [S, D]) for the proposal positions (l = -inf where the
    density fails).
    Returns (theta, logl, grad, accepted [S] bool, dH [S] = H1 - H0)."""
    theta = np.asarray(theta, np.float64)
    logl = np.asarray(logl, np.float64)
    m_inv = np.asarray(m_inv, np.float64)[None, :]
    p = np.asarray(z, np.float64) / np.sqrt(m_inv)
    h0 = -logl + 0.5 * np.sum(m_inv * p * p, axis=1)
    x, p, l1, g, inside = leapfrog(theta, p, grad, eps, m_inv, n_leapfrog, logl_grad, lo, hi)
    if n_leapfrog == 0:
        l1, g = logl, np.asarray(grad, np.float64)
    h1 = -l1 + 0.5 * np.sum(m_inv * p * p, axis=1)
    h1 = np.where(inside, h1, np.inf)
    dh = h1 - h0
    acc = np.asarray(logu) < -dh          # NaN compares false: rejected
    theta_new = np.where(acc[:, None], x, theta)
    logl_new = np.where(acc, l1, logl)
    grad_new = np.where(acc[:, None], g, grad)
    return theta_new, logl_new, grad_new, acc, dh


def gaussian_target(mu, prec):
    """l(theta) = -1/2 (theta - mu)^T prec (theta - mu) and its gradient."""
    mu = np.asarray(mu, np.float64)
    prec = np.asarray(prec, np.float64)

    def f(x):
        d = x - mu
        return -0.5 * np.einsum("si,ij,sj->s", d, prec, d), -d @ prec

    return f


def oracle_target(d, orc):
    """l(theta) = logL of dataset d (free parameters theta) from the oracle's
    filter, its gradient by complex-step differentiation of that filter."""
    free = np.asarray(d.free_idx)

    def f(x):
        c = d.to_canon(x)
        ll, st = orc.loglike(d, c)
        g = orc.grad_cs(d, c, which=free)
        ll = np.where(st == 0, ll, -np.inf)
        g = np.where((st == 0)[:, None], g, 0.0)
        return ll, g

    return f
