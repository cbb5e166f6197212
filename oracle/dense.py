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
      (G = identity for the per-pulsar models, Hellings-Downs for the joint)
  OU DM delay (model 4):           c c' v_d exp(-gamma_d |s - s'|),
      c = (1400 MHz / nu)^2 the chromatic factor of each TOA
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
    k = 6 if d.model == 4 else 4
    G = hd_closed_form(d.pos) if d.model == 3 else np.eye(P)
    vc = common_var(c[k * P], c[k * P + 1], d.t_span)
    Kc = np.exp(-lam * tau) * G[psr[:, None], psr[None, :]] * vc
    Cm += Kc
    parts[k * P] = 2 * LN10 * Kc
    parts[k * P + 1] = (np.log(1.0 / YEAR) + np.log(d.t_span) - 1.0 / (c[k * P + 1] - 1.0)) * Kc
    ss2 = d.sigma_s ** 2
    for q in range(P):
        sl = slice(int(d.off[q]), int(d.off[q + 1]))
        tq = t[sl]
        lsr, lgr, efac, leq = c[k * q:k * q + 4]
        gr = 10.0 ** lgr
        vr = 10.0 ** (2 * lsr) / (2 * gr)
        base, walk = _spin_k(tq, d.s_r, d.s_f, ss2)
        tq_tau = np.abs(tq[:, None] - tq[None, :])
        Kr = vr * np.exp(-gr * tq_tau)
        Rq = efac ** 2 * d.sigma[sl] ** 2 + 10.0 ** (2 * leq)
        Cm[sl, sl] += base + walk + Kr + np.diag(Rq)
        blocks = [2 * LN10 * Kr, -LN10 * (1.0 + gr * tq_tau) * Kr,
                  np.diag(2 * efac * d.sigma[sl] ** 2),
                  np.diag(2 * LN10 * 10.0 ** (2 * leq) * np.ones(tq.size))]
        if d.model == 4:
            lsd, lgd = c[k * q + 4:k * q + 6]
            gd = 10.0 ** lgd
            vd = 10.0 ** (2 * lsd) / (2 * gd)
            ch = (1400.0 / np.asarray(d.freq, np.float64)[sl]) ** 2
            Kd = vd * np.exp(-gd * tq_tau) * np.outer(ch, ch)
            Cm[sl, sl] += Kd
            blocks += [2 * LN10 * Kd, -LN10 * (1.0 + gd * tq_tau) * Kd]
        if with_parts:
            for j, blk in enumerate(blocks):
                full = np.zeros((N, N))
                full[sl, sl] = blk
                parts[k * q + j] = full
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


def state_cross_cov(d, c):
    """Prior covariances of the latent state at every TOA with every TOA's
    residual: K [nc, N, N], K[m, k, j] = Cov(x_m(t_k) of TOA k's pulsar, y_j),
    and the prior variances V [nc, N] of those state components. Components
    [r, f, a, g] (model 1: [r, f]; model 4: [r, f, a, g, m]); from the same
    covariance functions as
    covariance(), with the spin ones differentiated in the first time:
      Cov(f(s), r(s')) = s_f^2 s' + sigma_s^2 (s <= s' ? s s' - s^2/2 : s'^2/2),
      Var r(s) = s_r^2 + s_f^2 s^2 + sigma_s^2 s^3/3,  Var f(s) = s_f^2 + sigma_s^2 s."""
    c = np.asarray(c, np.float64)
    t = np.asarray(d.t, np.float64)
    N = t.size
    psr = np.repeat(np.arange(d.n_psr), np.diff(d.off))
    same = (psr[:, None] == psr[None, :]).astype(np.float64)
    ss2 = 10.0 ** (2 * c[0]) if d.model == 1 else d.sigma_s ** 2
    tk, tj = t[:, None], t[None, :]
    m = np.minimum(tk, tj)
    M = np.maximum(tk, tj)
    Kr = d.s_r ** 2 + d.s_f ** 2 * tk * tj + ss2 * m * m * (3 * M - m) / 6.0
    Kf = d.s_f ** 2 * tj + ss2 * np.where(tk <= tj, tk * tj - 0.5 * tk * tk, 0.5 * tj * tj)
    Vr = d.s_r ** 2 + d.s_f ** 2 * t * t + ss2 * t ** 3 / 3.0
    Vf = d.s_f ** 2 + ss2 * t
    if d.model == 1:
        return np.stack([Kr * same, Kf * same]), np.stack([Vr, Vf])
    P = d.n_psr
    k = 6 if d.model == 4 else 4
    tau = np.abs(tk - tj)
    gr = 10.0 ** c[1:k * P:k]
    vr = 10.0 ** (2 * c[0:k * P:k]) / (2 * gr)
    Ka = vr[psr][:, None] * np.exp(-gr[psr][:, None] * tau) * same
    G = hd_closed_form(d.pos) if d.model == 3 else np.eye(P)
    vc = common_var(c[k * P], c[k * P + 1], d.t_span)
    Kg = vc * G[psr[:, None], psr[None, :]] * np.exp(-(2 * np.pi / d.t_span) * tau)
    K = [Kr * same, Kf * same, Ka, Kg]
    V = [Vr, Vf, vr[psr], vc * np.diag(G)[psr]]
    if d.model == 4:
        # DM delay m at the reference frequency: residual j sees ch_j m(t_j),
        # so Cov(m(t_k), y_j) = ch_j v_d exp(-gamma_d |t_k - t_j|)
        gd = 10.0 ** c[5:k * P:k]
        vd = 10.0 ** (2 * c[4:k * P:k]) / (2 * gd)
        ch = (1400.0 / np.asarray(d.freq, np.float64)) ** 2
        K.append(vd[psr][:, None] * np.exp(-gd[psr][:, None] * tau) * ch[None, :] * same)
        V.append(vd[psr])
    return np.stack(K), np.stack(V)


def smooth(d, c):
    """Posterior mean and variance of each TOA's own pulsar state given all
    residuals, by Gaussian conditioning:
        E[x | y] = K C^-1 y,  Var[x | y] = V - diag(K C^-1 K^T)
    -> mean [N, nc], var [N, nc]."""
    Cm = covariance(d, c)
    y = np.asarray(d.y, np.float64)
    cf = sla.cho_factor(Cm, lower=True)
    alpha = sla.cho_solve(cf, y)
    K, V = state_cross_cov(d, c)
    mean = np.einsum("mkj,j->km", K, alpha)
    var = np.empty_like(mean)
    for m in range(K.shape[0]):
        var[:, m] = V[m] - np.einsum("kj,jk->k", K[m], sla.cho_solve(cf, K[m].T))
    return mean, var


def noise_posterior(d, c):
    """Posterior mean and variance of the white noise n = y - h.x at every
    TOA: E[n | y] = R C^-1 y and Var[n | y] = R - R^2 diag(C^-1), R the
    white variances (the same conditioning with Cov(n, y) = R)."""
    Cm = covariance(d, c)
    y = np.asarray(d.y, np.float64)
    c = np.asarray(c, np.float64)
    sig = np.asarray(d.sigma, np.float64)
    if d.model == 1:
        R = c[1] ** 2 * sig ** 2
    else:
        psr = np.repeat(np.arange(d.n_psr), np.diff(d.off))
        k = 6 if d.model == 4 else 4
        R = c[k * psr + 2] ** 2 * sig ** 2 + 10.0 ** (2 * c[k * psr + 3])
    cf = sla.cho_factor(Cm, lower=True)
    Ci = sla.cho_solve(cf, np.eye(y.size))
    return R * (Ci @ y), R - R * R * np.diag(Ci)


def smooth_mp(d, c, dps=40):
    """smooth() in mpmath arithmetic at dps decimal digits, for tiny inputs
    whose posterior variances are many decades below the prior ones (in
    fp64, V - diag(K C^-1 K^T) then cancels to a few digits). Covariance
    functions as in covariance() and state_cross_cov(), evaluated at high
    precision from the same fp64 inputs."""
    import mpmath as mp
    with mp.workdps(dps):
        c = [mp.mpf(float(v)) for v in np.asarray(c, np.float64)]
        t = [mp.mpf(float(v)) for v in d.t]
        y = mp.matrix([mp.mpf(float(v)) for v in d.y])
        sig = [mp.mpf(float(v)) for v in d.sigma]
        N = len(t)
        psr = np.repeat(np.arange(d.n_psr), np.diff(d.off))
        sr, sf = mp.mpf(float(d.s_r)), mp.mpf(float(d.s_f))
        if d.model == 1:
            ss2 = mp.mpf(10) ** (2 * c[0])
        else:
            ss2 = mp.mpf(float(d.sigma_s)) ** 2
            P = d.n_psr
            gr = [mp.mpf(10) ** c[4 * q + 1] for q in range(P)]
            vr = [mp.mpf(10) ** (2 * c[4 * q]) / (2 * gr[q]) for q in range(P)]
            G = hd_closed_form(d.pos) if d.model == 3 else np.eye(P)
            A, gam = c[4 * P], c[4 * P + 1]
            fyr, T = 1 / mp.mpf(YEAR), mp.mpf(float(d.t_span))
            vc = mp.mpf(10) ** (2 * A) * fyr ** (gam - 3) * T ** (gam - 1) / (
                12 * mp.pi ** 2 * (gam - 1))
            lam = 2 * mp.pi / T

        def k_spin(a, b):  # Cov(r(a), r(b)), Cov(f(a), r(b))
            mn, mx = min(a, b), max(a, b)
            kr = sr ** 2 + sf ** 2 * a * b + ss2 * mn * mn * (3 * mx - mn) / 6
            kf = sf ** 2 * b + ss2 * (a * b - a * a / 2 if a <= b else b * b / 2)
            return kr, kf

        nc = 2 if d.model == 1 else 4
        K = [mp.matrix(N, N) for _ in range(nc)]
        Cm = mp.matrix(N, N)
        for i in range(N):
            for j in range(N):
                pi_, pj = int(psr[i]), int(psr[j])
                comp = [mp.mpf(0)] * nc
                if pi_ == pj:
                    comp[0], comp[1] = k_spin(t[i], t[j])
                if d.model != 1:
                    tau = abs(t[i] - t[j])
                    if pi_ == pj:
                        comp[2] = vr[pi_] * mp.exp(-gr[pi_] * tau)
                    comp[3] = vc * mp.mpf(float(G[pi_, pj])) * mp.exp(-lam * tau)
                for m in range(nc):
                    K[m][i, j] = comp[m]
                # y = r + a + g + white: Cov(y_i, y_j) = Cov(r_i + a_i + g_i, y_j)
                Cm[i, j] = comp[0] + (comp[2] + comp[3] if d.model != 1 else 0)
            pq = int(psr[i])
            if d.model == 1:
                Cm[i, i] += c[1] ** 2 * sig[i] ** 2
            else:
                Cm[i, i] += c[4 * pq + 2] ** 2 * sig[i] ** 2 + mp.mpf(10) ** (2 * c[4 * pq + 3])
        Ci = mp.inverse(Cm)
        alpha = Ci * y
        mean = np.empty((N, nc))
        var = np.empty((N, nc))
        for m in range(nc):
            km = K[m] * alpha
            W = K[m] * Ci
            for k in range(N):
                pq = int(psr[k])
                if m == 0:
                    v0 = sr ** 2 + sf ** 2 * t[k] ** 2 + ss2 * t[k] ** 3 / 3
                elif m == 1:
                    v0 = sf ** 2 + ss2 * t[k]
                elif m == 2:
                    v0 = vr[pq]
                else:
                    v0 = vc * mp.mpf(float(G[pq, pq]))
                s = mp.mpf(0)
                for j in range(N):
                    s += W[k, j] * K[m][k, j]
                mean[k, m] = float(km[k])
                var[k, m] = float(v0 - s)
        return mean, var
