"""Pins of the CPU oracle against things other than itself: the dense Gaussian
likelihood (its plain definition), Van Loan's matrix exponential, textbook
special cases, Hellings-Downs quadrature over the sky, the power-law variance
integral and filter invariants. CPU only."""
import numpy as np
import pytest
import scipy.integrate as si
import scipy.linalg as sla

import pta_inputs as pi

pytestmark = []


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(np.abs(np.asarray(b)), 1.0)


# ----------------------------------------------------------- small datasets
def small_spin(seed=5, n=120, T_years=3.0):
    return pi.make_spin("t1", n_toa=n, T_years=T_years, seed=seed)


def small_pta(seed=7, counts=(40, 25, 60), model=pi.M_PSR4):
    return pi.make_pta("t2", n_psr=len(counts), counts=list(counts), seed=seed, model=model)


def moderate_theta(d, S, seed):
    """Samples away from the ill-conditioned corner of the dense form."""
    th = pi.sample_theta(d, S, seed)
    if d.model == pi.M_SPIN:
        th[:, 0] = np.minimum(th[:, 0], -15.5)
    return th


# ------------------------------------------------ 1. dense Gaussian parity
@pytest.mark.parametrize("model", [1, 2, 3])
def test_filter_equals_dense_gaussian(oracle_mod, model):
    from oracle import dense
    if model == 1:
        d = small_spin()
    else:
        d = small_pta(model=model)
    c = d.to_canon(moderate_theta(d, 6, 11))
    c = np.vstack([c, d.truth])
    ll, st = oracle_mod.loglike(d, c)
    assert (st == 0).all()
    ref = np.array([dense.loglike(d, ci) for ci in c])
    assert rel(ll, ref).max() < 1e-10, (ll, ref)


# ------------------------------------------- 2. discretisation vs Van Loan
def van_loan(A, LLt, dt):
    n = A.shape[0]
    M = np.zeros((2 * n, 2 * n))
    M[:n, :n] = -A
    M[:n, n:] = LLt
    M[n:, n:] = A.T
    E = sla.expm(M * dt)
    F = E[n:, n:].T
    Q = F @ E[:n, n:]
    return F, 0.5 * (Q + Q.T)


def continuous_model(d, c):
    """Drift A and diffusion L L^T of the continuous-time model, written from
    the SDEs: dr = f dt, df = s dW, da = -g a dt + sr dW, dg = -lam g dt + sc dW."""
    lam = 2 * np.pi / d.t_span
    if d.model == 1:
        A = np.array([[0, 1.0], [0, 0]])
        return A, np.diag([0, 10.0 ** (2 * c[0])])
    P = d.n_psr
    from oracle.dense import common_var, hd_closed_form
    vc = common_var(c[4 * P], c[4 * P + 1], d.t_span)
    blocks_A, diffs = [], []
    for q in range(P if d.model == 3 else 1):
        gr = 10.0 ** c[4 * q + 1]
        A = np.zeros((4, 4))
        A[0, 1] = 1.0
        A[2, 2] = -gr
        A[3, 3] = -lam
        blocks_A.append(A)
        diffs.append(np.diag([0, d.sigma_s ** 2, 10.0 ** (2 * c[4 * q]), 2 * lam * vc]))
    A = sla.block_diag(*blocks_A)
    LLt = sla.block_diag(*diffs)
    if d.model == 3:
        G = hd_closed_form(d.pos)
        for a in range(P):
            for b in range(P):
                LLt[4 * a + 3, 4 * b + 3] = 2 * lam * vc * G[a, b]
    return A, LLt


@pytest.mark.parametrize("model", [1, 2, 3])
@pytest.mark.parametrize("dt", [0.0, 1e3, 3e5, 2e6, 3e7])
def test_discretisation_van_loan(oracle_mod, model, dt):
    d = small_spin() if model == 1 else small_pta(model=model)
    c = d.truth.copy()
    if model == 1:
        c[0] = -13.0
    else:
        c[0:4] = [-11.0, -7.3, 1.0, -7.0]
    F, Q, _ = oracle_mod.model_mats(d, c, 0, dt)
    A, LLt = continuous_model(d, c)
    Fv, Qv = van_loan(A, LLt, dt)
    np.testing.assert_allclose(F, Fv, rtol=1e-12, atol=1e-300)
    # Q entries span many decades; compare each against its own scale
    scale = np.sqrt(np.outer(np.diag(Qv), np.diag(Qv))) + 1e-300
    assert (np.abs(Q - Qv) / scale).max() < 1e-9
    if dt == 0.0:
        assert np.array_equal(F, np.eye(F.shape[0])) and not Q.any()


def test_ou_limits(oracle_mod):
    d = small_pta()
    c = d.truth.copy()
    c[0:2] = [-11.0, -8.0]
    gr = 1e-8
    vr = 10.0 ** (-22) / (2 * gr)
    # gamma dt << 1: Q -> sigma^2 dt ; gamma dt >> 1: Q -> v, F -> 0
    _, Q, _ = oracle_mod.model_mats(d, c, 0, 1.0)
    assert abs(Q[2, 2] - 1e-22 * 1.0) / (1e-22) < 1e-7
    F, Q, _ = oracle_mod.model_mats(d, c, 0, 1e11)
    assert F[2, 2] == 0.0 and abs(Q[2, 2] - vr) / vr < 1e-15


# ---------------------------------------------------- 3. special cases
def test_white_only_closed_form(oracle_mod):
    d = small_pta(counts=(30, 50))
    d.s_r = d.s_f = d.sigma_s = 0.0
    c = d.truth.copy()
    for q in range(2):
        c[4 * q] = -400.0     # sigma_red -> 0 (underflows to exactly 0)
    c[-2] = -400.0            # A_c -> 0
    ll, st = oracle_mod.loglike(d, c[None])
    R = np.concatenate([c[4 * q + 2] ** 2 * d.sigma[d.off[q]:d.off[q + 1]] ** 2
                        + 10.0 ** (2 * c[4 * q + 3]) for q in range(2)])
    ref = np.sum(-0.5 * (np.log(2 * np.pi * R) + d.y ** 2 / R))
    assert st[0] == 0 and rel(ll[0], ref) < 1e-13


def test_single_toa(oracle_mod):
    d = small_pta(counts=(1,))
    c = d.truth
    ll, _ = oracle_mod.loglike(d, c[None])
    t1 = d.t[0]
    from oracle.dense import common_var
    vr = 10.0 ** (2 * c[0]) / (2 * 10.0 ** c[1])
    var = (d.s_r ** 2 + d.s_f ** 2 * t1 ** 2 + d.sigma_s ** 2 * t1 ** 3 / 3 + vr
           + common_var(c[4], c[5], d.t_span) + c[2] ** 2 * d.sigma[0] ** 2 + 10.0 ** (2 * c[3]))
    ref = -0.5 * (np.log(2 * np.pi * var) + d.y[0] ** 2 / var)
    assert rel(ll[0], ref) < 1e-14


def test_empty_pulsar_contributes_zero(oracle_mod):
    d = small_pta(counts=(30, 0, 20))
    dd = pi.subset(d, [0, 2])
    c = d.to_canon(pi.sample_theta(d, 3, 4))
    cc = np.hstack([c[:, 0:4], c[:, 8:12], c[:, -2:]])
    a, _ = oracle_mod.loglike(d, c)
    b, _ = oracle_mod.loglike(dd, cc)
    assert rel(a, b).max() < 1e-14


# ---------------------------------------------------- 4. structure
def test_additivity_over_pulsars(oracle_mod):
    d = small_pta(counts=(30, 45, 12, 60))
    c = d.to_canon(pi.sample_theta(d, 4, 3))
    tot, _, per = oracle_mod.loglike(d, c, per_psr=True)
    parts = []
    for q in range(4):
        dq = pi.subset(d, [q])
        cq = np.hstack([c[:, 4 * q:4 * q + 4], c[:, -2:]])
        parts.append(oracle_mod.loglike(dq, cq)[0])
    parts = np.array(parts).T
    assert rel(tot, parts.sum(1)).max() < 1e-13
    assert rel(per, parts).max() < 1e-14


def test_joint_single_pulsar_equals_per_pulsar(oracle_mod):
    d2 = small_pta(counts=(50,))
    d3 = small_pta(counts=(50,), model=pi.M_JOINT)
    c = d2.to_canon(pi.sample_theta(d2, 4, 9))
    a, _ = oracle_mod.loglike(d2, c)
    b, _ = oracle_mod.loglike(d3, c)
    assert rel(a, b).max() < 1e-12


def test_joint_without_common_is_sum_of_pulsars(oracle_mod):
    d2 = small_pta(counts=(20, 35, 15))
    d3 = small_pta(counts=(20, 35, 15), model=pi.M_JOINT)
    c = d2.to_canon(pi.sample_theta(d2, 3, 9))
    c[:, -2] = -400.0  # v_c -> 0: the HD coupling carries no variance
    a, _ = oracle_mod.loglike(d2, c)
    b, _ = oracle_mod.loglike(d3, c)
    assert rel(a, b).max() < 1e-12


@pytest.mark.parametrize("model", [2, 3])
def test_pulsar_permutation(oracle_mod, model):
    d = small_pta(counts=(20, 35, 15, 28), model=model)
    c = d.to_canon(pi.sample_theta(d, 3, 21))
    perm = [2, 0, 3, 1]
    dp = pi.subset(d, perm)
    cp = np.hstack([c[:, 4 * q:4 * q + 4] for q in perm] + [c[:, -2:]])
    a, _ = oracle_mod.loglike(d, c)
    b, _ = oracle_mod.loglike(dp, cp)
    assert rel(a, b).max() < 1e-12


def test_tied_toas_order(oracle_mod):
    """Simultaneous TOAs of different pulsars: the joint result does not
    depend on which is processed first (pulsar relabelling flips the order)."""
    d = small_pta(counts=(15, 15), model=pi.M_JOINT)
    d.t[15:] = d.t[:15]  # pulsar 1 observed at exactly pulsar 0's times
    c = d.to_canon(pi.sample_theta(d, 3, 2))
    dp = pi.subset(d, [1, 0])
    cp = np.hstack([c[:, 4:8], c[:, 0:4], c[:, -2:]])
    a, _ = oracle_mod.loglike(d, c)
    b, _ = oracle_mod.loglike(dp, cp)
    idx, psr = oracle_mod.merged_order(d)
    assert (psr[:2] == [0, 1]).all() and d.t[idx[0]] == d.t[idx[1]]
    assert rel(a, b).max() < 1e-12


def test_unit_rescaling(oracle_mod):
    """Measuring time residuals in other units: scaling y, sigma, EQUAD,
    s_r, s_f, sigma_s, sigma_red and sqrt(v_c) by k gives logL - N ln k."""
    d = small_pta(counts=(30, 40))
    c = d.to_canon(pi.sample_theta(d, 3, 5))
    k = 7.3
    ds = pi.make_pta("t2", n_psr=2, counts=[30, 40], seed=7)
    ds.y = d.y * k
    ds.sigma = d.sigma * k
    ds.s_r, ds.s_f, ds.sigma_s = d.s_r * k, d.s_f * k, d.sigma_s * k
    cs = c.copy()
    for q in range(2):
        cs[:, 4 * q] += np.log10(k)
        cs[:, 4 * q + 3] += np.log10(k)
    cs[:, -2] += np.log10(k)
    a, _ = oracle_mod.loglike(d, c)
    b, _ = oracle_mod.loglike(ds, cs)
    assert rel(b, a - d.n_toa * np.log(k)).max() < 1e-12


@pytest.mark.parametrize("model", [1, 2, 3])
def test_covariance_stays_spd(oracle_mod, model):
    d = small_spin() if model == 1 else small_pta(model=model)
    c = d.to_canon(pi.sample_theta(d, 1, 8))[0]
    tr = oracle_mod.trace(d, c, 0)
    assert tr["status"] == 0
    for Pk in list(tr["Pf"]) + list(tr["Pp"]):
        assert np.array_equal(Pk, Pk.T) or np.abs(Pk - Pk.T).max() <= 1e-15 * np.abs(Pk).max()
        np.linalg.cholesky(Pk + 0.0)  # raises unless positive-definite
    assert (tr["S"] > 0).all()
    # the trace's accumulated innovations reproduce the returned logL
    ll = np.sum(-0.5 * (np.log(2 * np.pi) + np.log(tr["S"]) + tr["e"] ** 2 / tr["S"]))
    assert rel(ll, tr["ll"]) < 1e-12


# ---------------------------------------------------- 5. HD and power law
def hd_quadrature(zeta, n=400):
    """Overlap reduction function by quadrature over GW directions:
    3/2 * <sum_A F^A_a F^A_b> over the sphere with
    F^A = 1/2 p^i p^j e^A_ij / (1 + Omega.p)."""
    pa = np.array([0.0, 0.0, 1.0])
    pb = np.array([np.sin(zeta), 0.0, np.cos(zeta)])
    x, w = np.polynomial.legendre.leggauss(n)
    phi = (np.arange(2 * n) + 0.5) * np.pi / n
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    om = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1)
    m = np.stack([np.sin(ph), -np.cos(ph), np.zeros_like(ph)], -1)
    nn = np.cross(om, m)
    def resp(p):
        den = 1.0 + om @ p
        mp, np_ = m @ p, nn @ p
        return 0.5 * (mp ** 2 - np_ ** 2) / den, 0.5 * (2 * mp * np_) / den
    Fa, Fb = resp(pa), resp(pb)
    integrand = Fa[0] * Fb[0] + Fa[1] * Fb[1]
    avg = (integrand * w[:, None]).sum() * (np.pi / n) / (4 * np.pi)
    return 1.5 * avg


@pytest.mark.parametrize("deg", [10.0, 49.0, 82.5, 90.0, 120.0, 150.0, 180.0])
def test_hd_against_sky_quadrature(oracle_mod, deg):
    z = np.radians(deg)
    pos = np.array([[0, 0, 1.0], [np.sin(z), 0, np.cos(z)]])
    G = oracle_mod.hd(pos)
    assert abs(G[0, 1] - hd_quadrature(z)) < 2e-5
    assert G[0, 0] == 1.0 and G[1, 1] == 1.0


def test_hd_known_values(oracle_mod):
    def at(deg):
        z = np.radians(deg)
        return oracle_mod.hd(np.array([[0, 0, 1.0], [np.sin(z), 0, np.cos(z)]]))[0, 1]
    assert abs(at(1e-9) - 0.5) < 1e-12
    assert abs(at(180.0) - 0.25) < 1e-12
    # 90 deg: x = 1/2 -> 3/4 ln(1/2) + 3/8
    assert abs(at(90.0) - (0.75 * np.log(0.5) + 0.375)) < 1e-12
    # minimum where d/dx (3/2 x ln x - x/4) = 0 -> x = exp(-5/6)
    xm = np.exp(-5.0 / 6.0)
    zm = np.degrees(np.arccos(1 - 2 * xm))
    vals = [at(zm + e) for e in (-0.01, 0.0, 0.01)]
    assert vals[1] < vals[0] and vals[1] < vals[2]
    assert abs(vals[1] - (-1.5 * xm + 0.5)) < 1e-12 and abs(vals[1] + 0.151897) < 1e-6


def test_hd_positive_definite(oracle_mod):
    d = pi.make_config("cfg3")
    G = oracle_mod.hd(d.pos)
    assert np.allclose(G, G.T)
    assert np.linalg.eigvalsh(G).min() > 0


@pytest.mark.parametrize("la,g", [(-15.0, 13 / 3), (-14.0, 2.5), (-13.5, 5.5)])
def test_power_law_variance(oracle_mod, la, g):
    T = 12 * pi.YEAR
    fyr = 1 / pi.YEAR
    psd = lambda f: 10 ** (2 * la) / (12 * np.pi ** 2) * fyr ** (g - 3) * f ** (-g)
    # substitute f = e^u for a well-behaved integrand
    val, err = si.quad(lambda u: psd(np.exp(u)) * np.exp(u), np.log(1 / T), np.log(1 / T) + 60,
                       epsabs=0, epsrel=1e-13, limit=400)
    v = oracle_mod.common_variance(la, g, T)
    assert abs(v - val) / val < 1e-10
    if la == -15.0:
        assert abs(np.sqrt(v) - 1.0e-7) / 1e-7 < 0.01


@pytest.mark.parametrize("model", [2, 4])
def test_common_amplitude_and_index_act_through_the_variance(oracle_mod, model):
    """log10 A and gamma of the common process enter the model only through
    its variance v_c = A^2 f_yr^(gamma - 3) T^(gamma - 1) / (12 pi^2 (gamma - 1))
    (the power-law common process of the Statement of Need, mapped as in
    reading R5), so dlogL/dgamma = dlogL/dlog10A (ln f_yr + ln T -
    1 / (gamma - 1)) / (2 ln 10) for every sample: the identity by which the
    GPU tangent sweeps take both derivatives from one tangent. Checked on the
    oracle's complex-step derivatives, which take the two separately."""
    if model == 2:
        d = small_pta(counts=(40, 25, 33))
        per = 4
    else:
        d = pi.make_pta_dm("t4", n_psr=3, counts=[40, 25, 33], seed=8)
        per = 6
    c = d.to_canon(moderate_theta(d, 3, 23))
    ia, ig = per * d.n_psr, per * d.n_psr + 1
    g = oracle_mod.grad_cs(d, c, which=[ia, ig])
    gam = c[:, ig]
    fac = (np.log(1.0 / pi.YEAR) + np.log(d.t_span) - 1.0 / (gam - 1.0)) / (2.0 * np.log(10.0))
    assert np.all(np.abs(g[:, 0]) > 0)
    assert np.allclose(g[:, 1], g[:, 0] * fac, rtol=1e-9, atol=0)


# ---------------------------------------------------- 6. gradient
@pytest.mark.parametrize("model", [1, 2, 3])
def test_complex_step_gradient_vs_dense(oracle_mod, model):
    from oracle import dense
    d = small_spin(n=60) if model == 1 else small_pta(counts=(25, 18, 30), model=model)
    c = d.to_canon(moderate_theta(d, 2, 17))
    g = oracle_mod.grad_cs(d, c)
    for s in range(c.shape[0]):
        gd = dense.grad(d, c[s])
        scale = np.abs(gd).max()
        assert (np.abs(g[s] - gd) / (np.abs(gd) + 1e-3 * scale)).max() < 1e-9


def test_complex_step_vs_central_fd(oracle_mod):
    d = small_pta(counts=(80, 40))
    c = d.to_canon(pi.sample_theta(d, 2, 23))
    g = oracle_mod.grad_cs(d, c)
    h = 1e-6
    for j in range(c.shape[1]):
        cp, cm = c.copy(), c.copy()
        cp[:, j] += h
        cm[:, j] -= h
        fd = (oracle_mod.loglike(d, cp)[0] - oracle_mod.loglike(d, cm)[0]) / (2 * h)
        assert (np.abs(fd - g[:, j]) <= 1e-5 * np.maximum(np.abs(g[:, j]), 1.0)).all()


# ---------------------------------------------------- 7. failure flags
def test_status_flags(oracle_mod):
    d = small_pta(counts=(10, 12))
    c = np.tile(d.truth, (3, 1))
    c[1, 2] = np.nan
    ll, st = oracle_mod.loglike(d, c)
    assert st[0] == 0 and st[1] == 2 and ll[1] == -np.inf
    dz = small_pta(counts=(10, 12))
    dz.s_r = dz.s_f = dz.sigma_s = 0.0
    cz = d.truth.copy()
    cz[[0, 4]] = -400.0
    cz[[2, 6]] = 0.0
    cz[[3, 7]] = -400.0
    cz[-2] = -400.0
    ll, st = oracle_mod.loglike(dz, cz[None])
    assert st[0] == 1 and ll[0] == -np.inf


# ---------------------------------------------------- 8. generator
def test_generator_is_deterministic():
    a = pi.make_config("cfg2")
    b = pi.make_config("cfg2")
    for f in ("t", "y", "sigma", "off", "pos", "truth"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    assert np.array_equal(pi.sample_theta(a, 8, 1), pi.sample_theta(b, 8, 1))
    assert a.n_psr == 47 and a.counts.min() >= 200 and a.counts.max() <= 2000
    for q in range(a.n_psr):
        assert np.all(np.diff(a.t[a.off[q]:a.off[q + 1]]) > 0)
