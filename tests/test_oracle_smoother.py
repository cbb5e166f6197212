"""Pins of the oracle's Rauch-Tung-Striebel smoother (the latent-state
posteriors that track the realised noise; paper: Summary, Statement of Need)
against its plain definition, Gaussian conditioning on the full TOA
covariance, and against identities and invariants of the posterior. CPU only.

The fp64 dense conditional V - diag(K C^-1 K^T) cancels to a few digits when
the posterior variance lies many decades below the prior one (the spin
frequency of the spin-only model), so the tightest pin is the same
conditioning in 40-digit arithmetic."""
import numpy as np
import pytest

import pta_inputs as pi


def spin(n=30, seed=5):
    return pi.make_spin("t1", n_toa=n, seed=seed)


def pta(counts, model=pi.M_PSR4, seed=31):
    return pi.make_pta("t2", n_psr=len(counts), counts=list(counts), seed=seed, model=model)


def err_mean(m, ref_m, ref_v):
    """Mean error in units of the posterior standard deviation."""
    return np.max(np.abs(m - ref_m) / np.sqrt(ref_v), initial=0.0)


def err_var(v, ref_v):
    return np.max(np.abs(v - ref_v) / ref_v, initial=0.0)


@pytest.mark.parametrize("model", [1, 2, 3])
def test_smoother_equals_high_precision_conditioning(oracle_mod, model):
    from oracle import dense
    d = spin() if model == 1 else pta([8, 12, 1], model=model)
    c = d.to_canon(pi.sample_theta(d, 3, 7))
    m, v, st = oracle_mod.smooth(d, c)
    assert (st == 0).all()
    for s in range(len(c)):
        em, ev = dense.smooth_mp(d, c[s])
        assert (ev > 0).all()
        assert err_mean(m[s], em, ev) < 1e-11
        assert err_var(v[s], ev) < 1e-11


@pytest.mark.parametrize("model", [2, 3])
def test_smoother_equals_fp64_conditioning(oracle_mod, model):
    """Larger streams, where only the fp64 conditional is affordable (the
    per-pulsar and joint models keep their posterior within a few decades of
    the prior, so fp64 conditioning keeps about 11 digits)."""
    from oracle import dense
    d = pta([40, 25, 0, 60], model=model, seed=7)
    c = d.to_canon(pi.sample_theta(d, 3, 11))
    m, v, st = oracle_mod.smooth(d, c)
    assert (st == 0).all()
    for s in range(len(c)):
        dm, dv = dense.smooth(d, c[s])
        assert err_mean(m[s], dm, dv) < 1e-9
        assert err_var(v[s], dv) < 1e-9


def test_dm_smoother_equals_fp64_conditioning(oracle_mod):
    """Model 4 (state r, f, a, g, m, each TOA seeing the DM delay through
    its chromatic factor): the RTS smoother of the 5-state filter against
    Gaussian conditioning with the dense DM covariance."""
    from oracle import dense
    d = pi.make_pta_dm("t", n_psr=3, counts=[40, 0, 60], seed=69)
    c = d.to_canon(pi.sample_theta(d, 3, 12))
    m, v, st = oracle_mod.smooth(d, c)
    assert (st == 0).all() and m.shape[-1] == 5
    for s in range(len(c)):
        dm, dv = dense.smooth(d, c[s])
        assert dm.shape[1] == 5
        assert err_mean(m[s], dm, dv) < 1e-9
        assert err_var(v[s], dv) < 1e-9


@pytest.mark.parametrize("model", [1, 2, 3])
def test_white_noise_posterior_identity(oracle_mod, model):
    """The white noise n_k = y_k - h.x_k has posterior mean R_k (C^-1 y)_k and
    variance R_k - R_k^2 (C^-1)_kk; the smoother's h.E[x_k|y] and
    h Cov[x_k|y] h^T must reproduce both (the latter pins the smoothed
    cross-covariances, which the component variances do not show)."""
    from oracle import dense
    if model == 1:
        d = spin(n=200, seed=8)
    else:
        d = pta([150, 90, 200], model=model, seed=9)
    c = d.to_canon(pi.sample_theta(d, 1, 12))[0]
    nm, nv = dense.noise_posterior(d, c)
    y = np.asarray(d.y)
    if model == 3:
        idx, psr = oracle_mod.merged_order(d)
        r = oracle_mod.smooth_stream(d, c)
        assert r["status"] == 0
        hx = np.empty(idx.size)
        hPh = np.empty(idx.size)
        for k, (j, q) in enumerate(zip(idx, psr)):
            h = np.zeros(4 * d.n_psr)
            h[[4 * q, 4 * q + 2, 4 * q + 3]] = 1.0
            hx[j] = h @ r["xs"][k]
            hPh[j] = h @ r["Ps"][k] @ h
    else:
        h = np.array([1.0, 0.0]) if model == 1 else np.array([1.0, 0.0, 1.0, 1.0])
        hx, hPh = [], []
        for q in range(d.n_psr):
            r = oracle_mod.smooth_stream(d, c, q)
            assert r["status"] == 0
            hx.append(r["xs"] @ h)
            hPh.append(np.einsum("i,kij,j->k", h, r["Ps"], h))
        hx, hPh = np.concatenate(hx), np.concatenate(hPh)
    scale = np.sqrt(nv)
    assert np.max(np.abs((y - hx) - nm) / scale) < 1e-8
    assert np.max(np.abs(hPh - nv) / nv) < 1e-8


def test_last_toa_is_filtered_and_smoothing_shrinks_variance(oracle_mod):
    d = pta([300, 1, 120])
    c = d.to_canon(pi.sample_theta(d, 2, 13))
    for s in range(2):
        for q in range(d.n_psr):
            tr = oracle_mod.trace(d, c[s], q)
            r = oracle_mod.smooth_stream(d, c[s], q)
            assert np.array_equal(r["xs"][-1], tr["x"][-1])
            assert np.array_equal(r["Ps"][-1], tr["Pf"][-1])
            fv = np.einsum("kii->ki", tr["Pf"])
            sv = np.einsum("kii->ki", r["Ps"])
            assert (sv <= fv * (1 + 1e-12)).all()
            assert (sv > 0).all()


def test_failed_filters_give_nan(oracle_mod):
    d = pta([10, 12, 8], seed=34)
    th = np.tile(d.truth, (3, 1))
    th[1, 5] = np.nan   # a parameter of pulsar 1: only its entries fail
    th[2, -1] = np.inf  # the common gamma: every pulsar fails
    dz = pta([6, 7], seed=48)
    dz.s_r = dz.s_f = dz.sigma_s = 0.0
    m, v, st = oracle_mod.smooth(d, d.to_canon(th))
    assert list(st) == [0, 2, 2]
    assert np.isnan(m[1, 10:22]).all() and np.isnan(v[1, 10:22]).all()
    assert np.isfinite(m[1, :10]).all() and np.isfinite(v[1, 22:]).all()
    assert np.isnan(m[2]).all() and np.isfinite(m[0]).all() and np.isfinite(v[0]).all()
    # every variance zero in pulsar 0 only: that pulsar's entries are NaN
    z = np.tile(dz.truth, (2, 1))
    z[0, [0, 2, 3]] = [-400.0, 0.0, -400.0]
    z[0, -2] = -400.0
    m, v, st = oracle_mod.smooth(dz, dz.to_canon(z))
    assert st[0] == 1 and st[1] == 0
    assert np.isnan(m[0, :6]).all() and np.isfinite(m[0, 6:]).all()
    # deterministic spin states (zero prior, no spin noise) smooth to exactly 0
    assert (m[1, :, :2] == 0).all() and (v[1, :, :2] == 0).all()


def test_spin_noise_after_a_long_gap(oracle_mod):
    """The regime where a plain covariance update loses digits: the
    strongest spin noise of the prior and a gap of about 800 days, after
    which the predicted residual variance exceeds the white variance by
    about 13 decades. The smoother must still match 40-digit conditioning."""
    import dataclasses
    from oracle import dense
    d = spin(n=200, seed=9)
    keep = np.r_[0:25, 75:100]
    d = dataclasses.replace(d, t=d.t[keep], y=d.y[keep], sigma=d.sigma[keep],
                            off=np.array([0, keep.size], np.int64))
    c = np.array([[d.hi[0], 1.0], [d.hi[0] - 0.5, 0.9]])
    m, v, st = oracle_mod.smooth(d, c)
    assert (st == 0).all()
    tr = oracle_mod.trace(d, c[0])
    assert tr["S"].max() / (c[0, 1] * d.sigma.min()) ** 2 > 1e12
    for s in range(len(c)):
        em, ev = dense.smooth_mp(d, c[s])
        assert err_mean(m[s], em, ev) < 1e-11
        assert err_var(v[s], ev) < 1e-11
