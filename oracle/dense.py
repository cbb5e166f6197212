"""The likelihood by its plain definition: log N(y; 0, C) with the full TOA
covariance C built from closed-form covariance functions and factorised by
Cholesky (the frequency-domain/dense formulation the paper contrasts the
Kalman filter with, Statement of Need). Used on tiny inputs to pin the
recursion in liboracle.so; shares no code with it.

TEST INFRASTRUCTURE ONLY.

Covariance functions (s = t - t0, t0 = 0 where the prior holds):
  spin [r, f] random walk with prior diag(s_r^2, s_f^2):
      s_r^2 + s_f^2 s s' + sigma_s^2 m^2 (3M - m) / 6,  m = min, M = max
  OU red noise (stationary):       v_r exp(-gamma_r |s - s'|)
  OU common process:               v_c exp(-lambda_c |s - s'|) * G_ab
      (G = identity for the per-pulsar model, Hellings-Downs for the joint)
  white:                           (EFAC^2 sigma_k^2 + EQUAD^2) delta
Gradient: d logL / d theta = 1/2 (alpha^T dC alpha - tr(C^-1 dC)),
alpha = C^-1 y (Rasmussen & Williams 2006, eq. 5.9).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

YEAR = 31557600.0
LN10 = np.log(10.0)


def hd_closed_form(pos):
    """Hellings-Downs matrix with the pulsar term on the diagonal."""
    pos = np.asarray(pos, np.float64)
    c = np.clip(pos @ pos.T, -1.0, 1.0)
    x = 0.5 * (1.0 - c)
    np.fill_diagonal(x, 0.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        xl = np.where(x > 0, x * np.log(np.where(x > 0, x, 1.0)), 0.0)
    return 1.5 * xl - 0.25 * x + 0.5 + 0.5 * np.eye(pos.shape[0])


def common_var(log10A, gam, T):
    fyr = 1.0 / YEAR
    return (10.0 ** (2 * log10A)) * fyr ** (gam - 3.0) * T ** (gam - 1.0) / (
        12 * np.pi ** 2 * (gam - 1.0))


def _spin_k(s, s_r, s_f, ss2):
    m = np.minimum.outer(s, s)
    M = np.maximum.outer(s, s)
    return s_r ** 2 + s_f ** 2 * np.outer(s, s), ss2 * m * m * (3 * M - m) / 6.0


def covariance(d, c, with_parts=False):
    """Dense covariance over all TOAs of dataset d (global TOA order) for the
    canonical vector c. With with_parts, also return dC/dc_j for every j."""
    c = np.asarray(c, np.float64)
    N = int(d.off[-1])
    t = np.asarray(d.t, np.float64)
    psr = np.repeat(np.arange(d.n_psr), np.diff(d.off))
    same = psr[:, None] == psr[None, :]
    tau = np.abs(t[:, None] - t[None, :])
    lam = 2 * np.pi / d.t_span
    parts = {}
    Cm = np.zeros((N, N))
    if d.model == 1:
        ss2 = 10.0 ** (2 * c[0])
        base, walk = _spin_k(t, d.s_r, d.s_f, ss2)
        R = c[1] ** 2 * d.sigma ** 2
        Cm = base + walk + np.diag(R)
        parts[0] = 2 * LN10 * walk
        parts[1] = np.diag(2 * c[1] * d.sigma ** 2)
        return (Cm, parts) if with_parts else Cm
    P = d.n_psr
    G = hd_closed_form(d.pos) if d.model == 3 else np.eye(P)
    vc = common_var(c[4 * P], c[4 * P + 1], d.t_span)
    Kc = np.exp(-lam * tau) * G[psr[:, None], psr[None, :]] * vc
    Cm += Kc
    parts[4 * P] = 2 * LN10 * Kc
    parts[4 * P + 1] = (np.log(1.0 / YEAR) + np.log(d.t_span) - 1.0 / (c[4 * P + 1] - 1.0)) * Kc
    ss2 = d.sigma_s ** 2
    for q in range(P):
        sl = slice(int(d.off[q]), int(d.off[q + 1]))
        tq = t[sl]
        lsr, lgr, efac, leq = c[4 * q:4 * q + 4]
        gr = 10.0 ** lgr
        vr = 10.0 ** (2 * lsr) / (2 * gr)
        base, walk = _spin_k(tq, d.s_r, d.s_f, ss2)
        tq_tau = np.abs(tq[:, None] - tq[None, :])
        Kr = vr * np.exp(-gr * tq_tau)
        Rq = efac ** 2 * d.sigma[sl] ** 2 + 10.0 ** (2 * leq)
        Cm[sl, sl] += base + walk + Kr + np.diag(Rq)
        if with_parts:
            for j, blk in enumerate([2 * LN10 * Kr,
                                     -LN10 * (1.0 + gr * tq_tau) * Kr,
                                     np.diag(2 * efac * d.sigma[sl] ** 2),
                                     np.diag(2 * LN10 * 10.0 ** (2 * leq) * np.ones(tq.size))]):
                full = np.zeros((N, N))
                full[sl, sl] = blk
                parts[4 * q + j] = full
    return (Cm, parts) if with_parts else Cm


def loglike(d, c):
    """log N(y; 0, C(c)) by Cholesky."""
    Cm = covariance(d, c)
    y = np.asarray(d.y, np.float64)
    L = np.linalg.cholesky(Cm)
    z = sla.solve_triangular(L, y, lower=True)
    return -0.5 * (y.size * np.log(2 * np.pi) + 2 * np.log(np.diag(L)).sum() + z @ z)


def grad(d, c):
    """d logL / d c for every canonical parameter (analytic dC)."""
    Cm, parts = covariance(d, c, with_parts=True)
    y = np.asarray(d.y, np.float64)
    cf = sla.cho_factor(Cm, lower=True)
    alpha = sla.cho_solve(cf, y)
    Ci = sla.cho_solve(cf, np.eye(y.size))
    g = np.zeros(len(c))
    for j, dC in parts.items():
        g[j] = 0.5 * (alpha @ dC @ alpha - np.sum(Ci * dC))
    return g
