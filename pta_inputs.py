"""Seeded synthetic PTA workloads: TOA cadences, per-TOA errors, sky positions,
simulated timing residuals, truths, prior boxes and parameter samples.

This module feeds both the oracle and the GPU library and holds none of the
likelihood's arithmetic: residual series are synthesised in the frequency
domain (sums of random sinusoids whose powers follow each process's spectrum)
and the gravitational-wave background is a sum of plane waves from random sky
directions seen through each pulsar's antenna pattern, so the Hellings-Downs
correlation emerges from geometry rather than from a formula. None of it
shares code with the Kalman filter's discretisation.

Workload shapes follow the paper's setting (Statement of Need: pulsars with
time-ordered TOAs; Functionality: red noise as OU, a common GWB, EFAC/EQUAD
white noise) at the five configurations the benchmarks use:
  cfg1  one pulsar, 500 TOAs over 10 yr, spin-only state [r, f]
  cfg2  47 pulsars, TOA counts log-uniform in [200, 2000], 12 yr, [r, f, a, g]
  cfg3  20 pulsars x 1000 TOAs, joint 80-state model with HD coupling
  cfg4  cfg2's data (gradient workload)
  cfg5  pulsars 0-9 of cfg2 with a 10-parameter free vector
and, for the per-pulsar model with dispersion-measure variations
(state [r, f, a, g, m]), cfg2dm: cfg2's pulsars and cadences observed in
four radio bands, with an OU DM delay per pulsar.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

YEAR = 31557600.0  # Julian year, s
M_SPIN, M_PSR4, M_JOINT, M_DM = 1, 2, 3, 4
NU_REF = 1400.0  # MHz: the DM delay state is the delay at this frequency
BANDS = np.array([430.0, 820.0, 1400.0, 2300.0])  # MHz
BAND_P = np.array([0.15, 0.35, 0.35, 0.15])
DM_LO = np.array([-14.0, -9.0])        # log10 sigma_dm, log10 gamma_dm
DM_HI = np.array([-10.0, -7.0])

# per-pulsar canonical parameters (models 2 and 3), then the two common ones
PSR_PARAM_NAMES = ("log10_sigma_red", "log10_gamma_red", "efac", "log10_equad")
PSR_LO = np.array([-14.0, -9.0, 0.8, -8.0])
PSR_HI = np.array([-10.0, -7.0, 1.2, -6.0])
COMMON_LO = np.array([-16.0, 2.0])     # log10 A, gamma (power law)
COMMON_HI = np.array([-13.0, 6.0])
COMMON_TRUTH = np.array([-14.5, 13.0 / 3.0])
SPIN_LO = np.array([-20.0, 0.8])       # model 1: log10 sigma_s, efac
SPIN_HI = np.array([-12.0, 1.2])

DATA_SEED = {"cfg1": 101, "cfg2": 102, "cfg3": 103, "cfg4": 102, "cfg5": 102, "cfg2dm": 102}
THETA_SEED = {"cfg1": 201, "cfg2": 202, "cfg3": 203, "cfg4": 204, "cfg5": 205, "cfg2dm": 206}
N_SAMPLES = {"cfg1": 64, "cfg2": 4096, "cfg3": 256, "cfg4": 1024, "cfg5": 65536, "cfg2dm": 4096}


@dataclass
class PTAData:
    name: str
    model: int
    n_psr: int
    off: np.ndarray          # int64 [P+1] CSR offsets
    t: np.ndarray            # float64 [N] s since epoch t0 = 0, ascending per pulsar
    y: np.ndarray            # float64 [N] residuals, s
    sigma: np.ndarray        # float64 [N] per-TOA 1-sigma error, s
    pos: np.ndarray | None   # float64 [P, 3] unit vectors
    t_span: float
    s_r: float = 1e-6
    s_f: float = 1e-14
    sigma_s: float = 1e-20
    truth: np.ndarray = field(default=None)     # canonical truth [C]
    lo: np.ndarray = field(default=None)        # prior box [C]
    hi: np.ndarray = field(default=None)
    free: np.ndarray = field(default=None)      # bool [C]
    freq: np.ndarray = field(default=None)      # float64 [N] radio frequency, MHz (model 4)

    @property
    def n_canon(self) -> int:
        if self.model == M_SPIN:
            return 2
        return (6 if self.model == M_DM else 4) * self.n_psr + 2

    @property
    def n_toa(self) -> int:
        return int(self.off[-1])

    @property
    def counts(self) -> np.ndarray:
        return np.diff(self.off)

    @property
    def free_idx(self) -> np.ndarray:
        return np.nonzero(self.free)[0].astype(np.int32)

    @property
    def n_free(self) -> int:
        return int(self.free.sum())

    def to_canon(self, theta: np.ndarray) -> np.ndarray:
        """Expand free parameters [S, D] to canonical vectors [S, C]."""
        theta = np.atleast_2d(np.asarray(theta, dtype=np.float64))
        c = np.tile(self.truth, (theta.shape[0], 1))
        c[:, self.free] = theta
        return c


# ------------------------------------------------------------------ helpers
def _cadence(rng, n, T):
    """n TOA times from t0 = 0 with exponential gaps of mean T/n."""
    if n == 0:
        return np.zeros(0)
    return np.cumsum(rng.exponential(T / n, size=n))


def _sigmas(rng, n, lo=5e-8, hi=2e-7):
    return 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), size=n)


def _sky(rng, P):
    v = rng.normal(size=(P, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _logfreq(T, nf, lo=1e-3, hi=1e3):
    edges = np.geomspace(lo / T, hi / T, nf + 1)
    return np.sqrt(edges[1:] * edges[:-1]), np.diff(edges)


def _synth(rng, t, psd, f, df):
    """Random-phase sinusoid sum with one-sided power psd(f) in bins df."""
    amp = np.sqrt(psd * df)
    a = rng.normal(size=f.size) * amp
    b = rng.normal(size=f.size) * amp
    ph = 2.0 * np.pi * np.outer(t, f)
    return np.cos(ph) @ a + np.sin(ph) @ b


def _red_series(rng, t, var, rate, T):
    """Lorentzian spectrum of a stationary series with variance var and
    correlation rate `rate`: 4 var rate / (rate^2 + (2 pi f)^2)."""
    f, df = _logfreq(T, 300)
    psd = 4.0 * var * rate / (rate ** 2 + (2 * np.pi * f) ** 2)
    return _synth(rng, t, psd, f, df)


def _spin_series(rng, t, sigma_s, T, dt=86400.0):
    """Integrated random walk in f sampled on a daily grid (Euler)."""
    n = int(np.ceil(max(t.max(), T) / dt)) + 2
    tg = np.arange(n) * dt
    f = sigma_s * np.concatenate([[0.0], np.cumsum(rng.normal(size=n - 1) * np.sqrt(dt))])
    r = np.concatenate([[0.0], np.cumsum(0.5 * (f[1:] + f[:-1]) * dt)])
    return np.interp(t, tg, r)


def _gwb(rng, t_list, pos, log10A, gam, T, ndir=64, nf=80):
    """Plane-wave GWB: each of ndir isotropic directions carries two
    polarisations with power-law spectra (above 1/T); each pulsar responds with
    F^A = 1/2 p^i p^j e^A_ij / (1 + Omega.p). A per-pulsar incoherent term of
    half the variance is added, so <r_a r_b> approaches var * (HD_ab + d_ab/2)."""
    fyr = 1.0 / YEAR
    edges = np.geomspace(1.0 / T, 200.0 / T, nf + 1)
    f = np.sqrt(edges[1:] * edges[:-1])
    df = np.diff(edges)
    psd = (10.0 ** (2 * log10A)) / (12 * np.pi ** 2) * fyr ** (gam - 3.0) * f ** (-gam)
    # directions and polarisation tensors
    om = _sky(rng, ndir)
    ref = np.where(np.abs(om[:, 2:3]) < 0.9, np.array([[0, 0, 1.0]]), np.array([[1.0, 0, 0]]))
    m = np.cross(om, ref)
    m /= np.linalg.norm(m, axis=1, keepdims=True)
    n = np.cross(om, m)
    psi = rng.uniform(0, np.pi, ndir)
    c, s = np.cos(2 * psi)[:, None], np.sin(2 * psi)[:, None]
    ep = np.einsum("di,dj->dij", m, m) - np.einsum("di,dj->dij", n, n)
    ec = np.einsum("di,dj->dij", m, n) + np.einsum("di,dj->dij", n, m)
    ep, ec = c[:, :, None] * ep + s[:, :, None] * ec, -s[:, :, None] * ep + c[:, :, None] * ec
    # coefficients of each (direction, polarisation) series
    amp = np.sqrt(psd * df * 1.5 / ndir)
    ca = rng.normal(size=(ndir, 2, f.size)) * amp
    cb = rng.normal(size=(ndir, 2, f.size)) * amp
    out = []
    for p, tp in enumerate(t_list):
        if tp.size == 0:
            out.append(np.zeros(0))
            continue
        pp = pos[p]
        den = 1.0 + om @ pp
        Fp = 0.5 * np.einsum("i,dij,j->d", pp, ep, pp) / den
        Fc = 0.5 * np.einsum("i,dij,j->d", pp, ec, pp) / den
        ph = 2.0 * np.pi * np.outer(tp, f)
        cos, sin = np.cos(ph), np.sin(ph)
        wa = Fp[:, None] * ca[:, 0] + Fc[:, None] * ca[:, 1]
        wb = Fp[:, None] * cb[:, 0] + Fc[:, None] * cb[:, 1]
        r = cos @ wa.sum(0) + sin @ wb.sum(0)
        r += _synth(rng, tp, 0.5 * psd, f, df)  # pulsar term
        out.append(r)
    return out


def _draw_psr_truth(rng, P):
    return rng.uniform(PSR_LO, PSR_HI, size=(P, 4))


# ---------------------------------------------------------------- datasets
def make_spin(name="cfg1", n_toa=500, T_years=10.0, seed=None, sigma=1e-7,
              log10_sigma_s=-18.0):
    """Model 1: one pulsar, state [r, f]; white noise sigma * EFAC."""
    rng = np.random.default_rng(DATA_SEED.get(name, 101) if seed is None else seed)
    T = T_years * YEAR
    t = _cadence(rng, n_toa, T)
    sig = np.full(n_toa, sigma)
    efac = rng.uniform(0.8, 1.2)
    s_r, s_f = 1e-6, 1e-14
    y = (rng.normal() * s_r + rng.normal() * s_f * t
         + _spin_series(rng, t, 10.0 ** log10_sigma_s, T)
         + efac * sig * rng.normal(size=n_toa))
    truth = np.array([log10_sigma_s, efac])
    return PTAData(name, M_SPIN, 1, np.array([0, n_toa], np.int64), t, y, sig, None,
                   T, s_r, s_f, 0.0, truth, SPIN_LO.copy(), SPIN_HI.copy(),
                   np.ones(2, bool))


def make_pta(name="cfg2", n_psr=47, n_range=(200, 2000), counts=None,
             T_years=12.0, seed=None, model=M_PSR4, common=COMMON_TRUTH):
    """Models 2 and 3: P pulsars, per-pulsar state [r, f, a, g]."""
    rng = np.random.default_rng(DATA_SEED.get(name, 102) if seed is None else seed)
    T = T_years * YEAR
    if counts is None:
        lo, hi = np.log10(n_range[0]), np.log10(n_range[1])
        counts = np.rint(10.0 ** rng.uniform(lo, hi, size=n_psr)).astype(np.int64)
    counts = np.asarray(counts, np.int64)
    pos = _sky(rng, n_psr)
    ptruth = _draw_psr_truth(rng, n_psr)
    ts = [_cadence(rng, int(n), T) for n in counts]
    gw = _gwb(rng, ts, pos, common[0], common[1], T)
    ys, sigs = [], []
    for p in range(n_psr):
        tp = ts[p]
        lsr, lgr, efac, leq = ptruth[p]
        gr = 10.0 ** lgr
        vr = 10.0 ** (2 * lsr) / (2 * gr)
        sig = _sigmas(rng, tp.size)
        w = np.sqrt((efac * sig) ** 2 + 10.0 ** (2 * leq)) * rng.normal(size=tp.size)
        y = (rng.normal() * 1e-6 + rng.normal() * 1e-14 * tp
             + _red_series(rng, tp, vr, gr, T) + gw[p] + w)
        ys.append(y)
        sigs.append(sig)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    truth = np.concatenate([ptruth.ravel(), common])
    lo = np.concatenate([np.tile(PSR_LO, n_psr), COMMON_LO])
    hi = np.concatenate([np.tile(PSR_HI, n_psr), COMMON_HI])
    return PTAData(name, model, n_psr, off, np.concatenate(ts), np.concatenate(ys),
                   np.concatenate(sigs), pos, T, 1e-6, 1e-14, 1e-20, truth, lo, hi,
                   np.ones(truth.size, bool))


def make_pta_dm(name="cfg2dm", n_psr=47, n_range=(200, 2000), counts=None, T_years=12.0,
                seed=None, common=COMMON_TRUTH):
    """Model 4: make_pta's pulsars (same draws, so the same cadences, errors,
    truths and residuals) observed at a radio frequency drawn per TOA from
    four bands, plus a DM delay per pulsar: an OU series with the Lorentzian
    spectrum of its (sigma_dm, gamma_dm), scaled by (NU_REF / nu)^2. Per
    pulsar parameters [log10 sigma_red, log10 gamma_red, EFAC, log10 EQUAD,
    log10 sigma_dm, log10 gamma_dm], then [log10 A, gamma]."""
    base = make_pta(name, n_psr=n_psr, n_range=n_range, counts=counts, T_years=T_years,
                    seed=seed, model=M_DM, common=common)
    rng = np.random.default_rng(7919 + (DATA_SEED.get(name, 102) if seed is None else seed))
    P, T = base.n_psr, base.t_span
    dtruth = rng.uniform(DM_LO, DM_HI, size=(P, 2))
    freq = rng.choice(BANDS, size=base.n_toa, p=BAND_P)
    y = base.y.copy()
    for p in range(P):
        a, b = int(base.off[p]), int(base.off[p + 1])
        lsd, lgd = dtruth[p]
        gd = 10.0 ** lgd
        vd = 10.0 ** (2 * lsd) / (2 * gd)
        y[a:b] += _red_series(rng, base.t[a:b], vd, gd, T) * (NU_REF / freq[a:b]) ** 2
    pt = base.truth[:4 * P].reshape(P, 4)
    truth = np.concatenate([np.hstack([pt, dtruth]).ravel(), base.truth[-2:]])
    lo = np.concatenate([np.tile(np.r_[PSR_LO, DM_LO], P), COMMON_LO])
    hi = np.concatenate([np.tile(np.r_[PSR_HI, DM_HI], P), COMMON_HI])
    return PTAData(name, M_DM, P, base.off, base.t, y, base.sigma, base.pos, T, base.s_r,
                   base.s_f, base.sigma_s, truth, lo, hi, np.ones(truth.size, bool), freq)


def subset(d: PTAData, psrs, name=None, free=None) -> PTAData:
    """Pulsars `psrs` of d (same data, same truths); optional free mask."""
    psrs = list(psrs)
    segs = [(d.off[p], d.off[p + 1]) for p in psrs]
    cnt = np.array([b - a for a, b in segs], np.int64)
    cat = lambda arr: np.concatenate([arr[a:b] for a, b in segs]) if segs else arr[:0]
    truth = np.concatenate([d.truth[4 * p:4 * p + 4] for p in psrs] + [d.truth[-2:]])
    lo = np.concatenate([d.lo[4 * p:4 * p + 4] for p in psrs] + [d.lo[-2:]])
    hi = np.concatenate([d.hi[4 * p:4 * p + 4] for p in psrs] + [d.hi[-2:]])
    fr = np.ones(truth.size, bool) if free is None else np.asarray(free, bool)
    return PTAData(name or d.name, d.model, len(psrs),
                   np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64),
                   cat(d.t), cat(d.y), cat(d.sigma),
                   None if d.pos is None else d.pos[psrs], d.t_span, d.s_r, d.s_f,
                   d.sigma_s, truth, lo, hi, fr)


def cfg5_free_mask(n_psr=10) -> np.ndarray:
    """Ten free parameters: all four of pulsar 0, the red-noise pair of
    pulsars 1 and 2, and the two common parameters; the rest fixed at truth."""
    m = np.zeros(4 * n_psr + 2, bool)
    m[[0, 1, 2, 3, 4, 5, 8, 9]] = True
    m[-2:] = True
    return m


def make_config(name: str) -> PTAData:
    if name == "cfg1":
        return make_spin("cfg1")
    if name in ("cfg2", "cfg4"):
        return make_pta(name)
    if name == "cfg3":
        return make_pta("cfg3", n_psr=20, counts=np.full(20, 1000), model=M_JOINT)
    if name == "cfg5":
        return subset(make_pta("cfg2"), range(10), "cfg5", cfg5_free_mask(10))
    if name == "cfg2dm":
        return make_pta_dm("cfg2dm")
    raise ValueError(name)


def sample_theta(d: PTAData, S: int, seed: int) -> np.ndarray:
    """S free-parameter vectors drawn uniformly in the prior box, [S, D]."""
    rng = np.random.default_rng(seed)
    lo, hi = d.lo[d.free], d.hi[d.free]
    return rng.uniform(lo, hi, size=(S, lo.size))


def theta_near_truth(d: PTAData, S: int, seed: int, scale=0.05) -> np.ndarray:
    """Samples in a small box (fraction `scale` of the prior width) around the
    truth, clipped to the prior: the high-likelihood region."""
    rng = np.random.default_rng(seed)
    lo, hi, tr = d.lo[d.free], d.hi[d.free], d.truth[d.free]
    w = (hi - lo) * scale
    return np.clip(tr + rng.uniform(-w, w, size=(S, tr.size)), lo, hi)


def theta_from_ensemble(ens: np.ndarray, S: int, seed: int, lo, hi, widen=(1.0,)) -> np.ndarray:
    """S parameter vectors from the Gaussian with the mean and covariance of
    an ensemble of posterior draws `ens` [n, D] (a pilot sampler's chains),
    in equal parts with the covariance scaled by each factor of `widen`
    squared, clipped to the prior box [lo, hi]: training and starting points
    where the posterior puts its mass."""
    rng = np.random.default_rng(seed)
    ens = np.asarray(ens, np.float64)
    mu = ens.mean(0)
    L = np.linalg.cholesky(np.cov(ens, rowvar=False) + 1e-30 * np.eye(ens.shape[1]))
    parts = []
    for i, w in enumerate(widen):
        n = S // len(widen) + (1 if i < S % len(widen) else 0)
        parts.append(mu + w * rng.standard_normal((n, mu.size)) @ L.T)
    return np.clip(np.concatenate(parts), lo, hi)


def mlp_weights(d_in: int, width: int, seed: int) -> np.ndarray:
    """Initial surrogate weights, packed as W1 [w, d], b1, W2 [w, w], b2,
    W3 [w, w], b3, W4 [w], b4: He-uniform weights U(-sqrt(6/fan_in), ...),
    zero biases, values representable in FP32."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, shape in ((d_in, (width, d_in)), (width, (width, width)), (width, (width, width))):
        lim = np.sqrt(6.0 / fan_in)
        parts += [rng.uniform(-lim, lim, size=shape).ravel(), np.zeros(width)]
    lim = np.sqrt(6.0 / width)
    parts += [rng.uniform(-lim, lim, size=width), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32).astype(np.float64)
