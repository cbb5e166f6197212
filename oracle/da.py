"""Reference Metropolis-Hastings and delayed-acceptance Metropolis-Hastings
(Christen & Fox 2005) with symmetric random-walk proposals, written as plain
per-chain loops.

TEST INFRASTRUCTURE ONLY.

Delayed acceptance, for a proposal y from x with cheap approximation lq~ of
the target lq:
  stage 1: accept with probability min(1, exp(lq~(y) - lq~(x)));
  stage 2 (only after stage 1 accepts): accept with probability
           min(1, exp((lq(y) - lq(x)) - (lq~(y) - lq~(x)))).
The chain targets exp(lq) exactly whatever the error of lq~, and the exact
target is evaluated only for stage-1 survivors. Uniform random numbers are
inputs, so the GPU driver and this reference can consume the same draws.
"""
from __future__ import annotations

import numpy as np


def mh(lq, x0, steps, eps, logu):
    """Plain random-walk MH. eps [T, d] proposal increments, logu [T]."""
    x = np.array(x0, np.float64)
    lx = lq(x)
    out = np.empty((steps, x.size))
    acc = 0
    for t in range(steps):
        y = x + eps[t]
        ly = lq(y)
        if logu[t] < ly - lx:
            x, lx = y, ly
            acc += 1
        out[t] = x
    return out, acc / steps


def da_mh(lq, lq_approx, x0, steps, eps, logu1, logu2):
    """Delayed-acceptance MH. Returns (chain, stage-1 rate, overall rate,
    number of exact evaluations)."""
    x = np.array(x0, np.float64)
    lx, ax = lq(x), lq_approx(x)
    out = np.empty((steps, x.size))
    n1 = n2 = n_exact = 0
    for t in range(steps):
        y = x + eps[t]
        ay = lq_approx(y)
        if logu1[t] < ay - ax:
            n1 += 1
            ly = lq(y)
            n_exact += 1
            if logu2[t] < (ly - lx) - (ay - ax):
                x, lx, ax = y, ly, ay
                n2 += 1
        out[t] = x
    return out, n1 / steps, n2 / steps, n_exact
