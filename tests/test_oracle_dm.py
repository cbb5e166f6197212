"""Pins of the oracle's per-pulsar model with DM variations (model 4: state
[r, f, a, g, m], m the DM delay at 1400 MHz as an OU process, seen at a
TOA of radio frequency nu through (1400 / nu)^2): the filter against the
dense Gaussian likelihood, complex-step gradients against the dense
analytic gradient, the limit of vanishing DM noise (model 2), the
single-band case with equal rates (two OU processes of one rate are one OU
process of the summed variance), and the frequency-scaling invariance.
CPU only."""
import dataclasses

import numpy as np
import pytest

import pta_inputs as pi


def small_dm(seed=41, counts=(40, 0, 25, 60)):
    return pi.make_pta_dm("t4", n_psr=len(counts), counts=list(counts), seed=seed)


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(np.abs(np.asarray(b)), 1.0)


def test_dm_filter_equals_dense_gaussian(oracle_mod):
    from oracle import dense
    d = small_dm()
    c = np.vstack([d.to_canon(pi.sample_theta(d, 5, 3)), d.truth])
    ll, st = oracle_mod.loglike(d, c)
    assert (st == 0).all()
    ref = np.array([dense.loglike(d, ci) for ci in c])
    assert rel(ll, ref).max() < 1e-10


@pytest.mark.parametrize("seed", [4, 17])
def test_dm_gradient_equals_dense(oracle_mod, seed):
    """Per component, the criterion of the other models' gradient pin:
    |g_j - g_dense,j| <= 1e-9 (|g_dense,j| + 1e-3 max|g_dense|), so a small
    component such as a DM-rate derivative is held to the same relative
    bar as the large ones (measured worst 2.2e-11)."""
    from oracle import dense
    d = small_dm(counts=(30, 20))
    c = d.to_canon(pi.sample_theta(d, 2, seed))
    g = oracle_mod.grad_cs(d, c)
    for s in range(2):
        ref = dense.grad(d, c[s])
        scale = np.abs(ref).max()
        assert (np.abs(g[s] - ref) / (np.abs(ref) + 1e-3 * scale)).max() < 1e-9


def model2_view(d):
    """The same data as the per-pulsar model without the DM state."""
    P = d.n_psr
    keep = np.concatenate([np.r_[6 * q:6 * q + 4] for q in range(P)] + [np.r_[6 * P:6 * P + 2]])
    return dataclasses.replace(d, model=pi.M_PSR4, truth=d.truth[keep], lo=d.lo[keep],
                               hi=d.hi[keep], free=np.ones(keep.size, bool), freq=None), keep


def test_vanishing_dm_noise_is_model2(oracle_mod):
    d = small_dm()
    d2, keep = model2_view(d)
    c = d.to_canon(pi.sample_theta(d, 4, 5))
    c[:, 4::6][:, :d.n_psr] = -40.0  # log10 sigma_dm of every pulsar
    ll4, _ = oracle_mod.loglike(d, c)
    ll2, _ = oracle_mod.loglike(d2, c[:, keep])
    assert rel(ll4, ll2).max() < 1e-12


def test_single_band_equal_rates_sum_variances(oracle_mod):
    """At nu = 1400 MHz with gamma_dm = gamma_red the state a + m is one OU
    process of variance v_r + v_d: the likelihood equals model 2's with
    sigma_red^2 -> sigma_red^2 + sigma_dm^2 (v = sigma^2 / 2 gamma)."""
    d = dataclasses.replace(small_dm(), freq=np.full(125, 1400.0))
    d2, keep = model2_view(d)
    c = d.to_canon(pi.sample_theta(d, 4, 6))
    P = d.n_psr
    c2 = c[:, keep].copy()
    for q in range(P):
        c[:, 6 * q + 5] = c[:, 6 * q + 1]
        s2 = 10.0 ** (2 * c[:, 6 * q]) + 10.0 ** (2 * c[:, 6 * q + 4])
        c2[:, 4 * q] = 0.5 * np.log10(s2)
    ll4, _ = oracle_mod.loglike(d, c)
    ll2, _ = oracle_mod.loglike(d2, c2)
    assert rel(ll4, ll2).max() < 1e-12


def test_frequency_scaling_invariance(oracle_mod):
    """nu -> k nu with sigma_dm -> k^2 sigma_dm leaves the DM delay at every
    TOA, hence the likelihood, unchanged."""
    d = small_dm()
    k = 1.7
    dk = dataclasses.replace(d, freq=d.freq * k)
    c = d.to_canon(pi.sample_theta(d, 4, 7))
    ck = c.copy()
    ck[:, 4:6 * d.n_psr:6] += 2 * np.log10(k)
    ll, _ = oracle_mod.loglike(d, c)
    llk, _ = oracle_mod.loglike(dk, ck)
    assert rel(ll, llk).max() < 1e-12
