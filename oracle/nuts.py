"""No-U-Turn Sampler transition (FP64 reference, one chain at a time): the
sampler the paper's posteriors were drawn with (Functionality, "Sampler
Integration"; figure caption: NUTS of Hoffman & Gelman 2014), here with
multinomial trajectory sampling and the generalised no-U-turn criterion
(Betancourt 2017), written recursively.

For a chain at theta0 (log-density l0, gradient g0), momentum
p0 = z / sqrt(m_inv), H = -l + 1/2 sum m_inv p^2, H0 at the start:

* a leaf is one leapfrog step (step v eps, v = +-1) from the end it grows
  from; its log weight is -H; it diverges when H - H0 > 1000, H is not a
  number, the position leaves the box [lo, hi] or l is not finite;
* a subtree of depth j > 0 is a subtree of depth j - 1 followed by another
  grown from its last leaf; if the first is invalid the second is not
  built. Merging (A then B in build order): W = logaddexp(W_A, W_B); the
  proposal is B's when u < exp(W_B - W) for this merge's uniform u (merges
  numbered 0, 1, ... in post-order within the top-level subtree of
  doubling j, u = u_sub[j, m]), else A's; rho = rho_A + rho_B; the merged
  subtree makes a U-turn unless (m_inv p_first) . rho > 0 and
  (m_inv p_last) . rho > 0, p_first the first leaf of A and p_last the last
  leaf of B; a U-turn or a divergence makes it invalid;
* the trajectory starts as {theta0} (W = -H0, rho = p0). Doubling j draws
  the direction dirs[j], grows a subtree of 2^j leaves from the trajectory
  end on that side, and stops if it is invalid. Otherwise its proposal
  replaces the trajectory's when u_top[j] < exp(W_sub - W_traj) (biased
  progressive sampling), W and rho are combined, the end moves, and the
  trajectory stops when it makes a U-turn (same criterion on its two ends)
  or after max_depth doublings.

The random numbers (z, dirs, u_top, u_sub) are inputs, so a transition is a
deterministic function of them.

TEST INFRASTRUCTURE ONLY: imported by tests, never by the product path.
"""
from __future__ import annotations

import numpy as np

DIVERGENCE = 1000.0


class _Tree:
    __slots__ = ("first", "last", "prop", "W", "rho", "valid", "n", "acc", "div")


def _leaf(state, v, eps, m_inv, lo, hi, h0, f):
    x, p, g = state
    p = p + 0.5 * v * eps * g
    x = x + v * eps * m_inv * p
    l, g1 = f(x[None, :])
    l, g1 = float(l[0]), g1[0]
    p = p + 0.5 * v * eps * g1
    inside = bool(np.all((x >= lo) & (x <= hi))) and np.isfinite(l)
    h = -l + 0.5 * float(np.sum(m_inv * p * p)) if inside else np.inf
    t = _Tree()
    t.first = t.last = (x, p, g1)
    t.prop = (x, l, g1)
    t.W = -h
    t.rho = p.copy()
    t.div = not (h - h0 <= DIVERGENCE)
    t.valid = not t.div
    t.n = 1
    t.acc = min(1.0, float(np.exp(h0 - h))) if np.isfinite(h) else 0.0
    return t


def _no_uturn(p_a, p_b, rho, m_inv):
    return float(np.dot(m_inv * p_a, rho)) > 0.0 and float(np.dot(m_inv * p_b, rho)) > 0.0


def _build(state, v, j, eps, m_inv, lo, hi, h0, f, u_sub_j, counter):
    if j == 0:
        return _leaf(state, v, eps, m_inv, lo, hi, h0, f)
    a = _build(state, v, j - 1, eps, m_inv, lo, hi, h0, f, u_sub_j, counter)
    if not a.valid:
        return a
    b = _build(a.last, v, j - 1, eps, m_inv, lo, hi, h0, f, u_sub_j, counter)
    t = _Tree()
    t.n = a.n + b.n
    t.acc = a.acc + b.acc
    t.div = b.div
    t.first, t.last = a.first, b.last
    if not b.valid:
        t.valid = False
        t.prop, t.W, t.rho = a.prop, a.W, a.rho
        return t
    m = counter[0]
    counter[0] += 1
    t.W = float(np.logaddexp(a.W, b.W))
    t.prop = b.prop if u_sub_j[m] < np.exp(b.W - t.W) else a.prop
    t.rho = a.rho + b.rho
    t.valid = _no_uturn(a.first[1], b.last[1], t.rho, m_inv)
    return t


def transition_one(theta0, l0, g0, eps, m_inv, lo, hi, z, dirs, u_top, u_sub, max_depth, f):
    """One chain. Returns (theta, l, g, depth, n_leapfrog, divergent,
    mean acceptance statistic over the leaves)."""
    m_inv = np.asarray(m_inv, np.float64)
    x0 = np.asarray(theta0, np.float64)
    p0 = np.asarray(z, np.float64) / np.sqrt(m_inv)
    g0 = np.asarray(g0, np.float64)
    h0 = -float(l0) + 0.5 * float(np.sum(m_inv * p0 * p0))
    left = right = (x0, p0, g0)
    prop = (x0, float(l0), g0)
    W = -h0
    rho = p0.copy()
    depth = n = 0
    acc = 0.0
    div = False
    for j in range(max_depth):
        v = int(dirs[j])
        start = right if v > 0 else left
        sub = _build(start, v, j, eps, m_inv, lo, hi, h0, f, u_sub[j], [0])
        n += sub.n
        acc += sub.acc
        if not sub.valid:
            div = sub.div
            break
        if u_top[j] < np.exp(sub.W - W):
            prop = sub.prop
        W = float(np.logaddexp(W, sub.W))
        rho = rho + sub.rho
        if v > 0:
            right = sub.last
        else:
            left = sub.last
        depth = j + 1
        if not _no_uturn(left[1], right[1], rho, m_inv):
            break
    return prop[0], prop[1], prop[2], depth, n, div, acc / max(n, 1)


def transition(theta, logl, grad, eps, m_inv, lo, hi, z, dirs, u_top, u_sub, max_depth, f):
    """S chains, each by transition_one. dirs [S, max_depth] (+-1), u_top
    [S, max_depth], u_sub [S, max_depth, 2^(max_depth-1)]."""
    S = np.asarray(theta).shape[0]
    out = [transition_one(theta[s], logl[s], grad[s], float(np.asarray(eps)[s]), m_inv, lo, hi,
                          z[s], dirs[s], u_top[s], u_sub[s], max_depth, f) for s in range(S)]
    th = np.array([o[0] for o in out])
    ll = np.array([o[1] for o in out])
    g = np.array([o[2] for o in out])
    depth = np.array([o[3] for o in out], np.int32)
    n = np.array([o[4] for o in out], np.int32)
    div = np.array([o[5] for o in out], bool)
    acc = np.array([o[6] for o in out])
    return th, ll, g, depth, n, div, acc


def draws(rng, S, D, max_depth):
    """The random inputs of one transition for S chains."""
    z = rng.normal(size=(S, D))
    dirs = np.where(rng.random((S, max_depth)) < 0.5, -1, 1).astype(np.int32)
    u_top = rng.random((S, max_depth))
    u_sub = rng.random((S, max_depth, max(1, 2 ** (max_depth - 1))))
    return z, dirs, u_top, u_sub
