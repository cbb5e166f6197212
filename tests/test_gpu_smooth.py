"""Parity of the HIP smoother (argus_smooth: for models 1 and 2 the
checkpointed filter pass followed by the modified Bryson-Frazier recursion,
E[x|y] = x - P lam and Cov[x|y] = P - P Lam P per TOA, either one wave per
(64-sample tile, pulsar) or in the time-parallel form whose reverse sweep
runs over chunks of each stream at once; for the DM model the same
recursion over the filtered 5-state filter) with the oracle's
Rauch-Tung-Striebel recursion, element by element, through the C ABI.

Tolerances: |mean_gpu - mean_ref| <= 1e-9 sd_ref and |var_gpu - var_ref| <=
1e-8 var_ref, sd_ref = sqrt(var_ref). Both sides are fp64 but follow
different algebra: each obtains the smoothed covariance by subtracting a
data-driven correction from a filtered or predicted one, so its rounding
error is relative to that larger covariance. Measured on the GPU over all
1024 samples of the 47-pulsar batch, every form of models 1 and 2 stays
within 8e-12 sd in the mean and 6e-11 in relative variance; the
time-parallel form's chained chunk summaries add no visible error. The
bounds keep the margin the DM model needs. Deterministic components (zero
variance) must match exactly."""
import numpy as np
import pytest

import pta_inputs as pi

pytestmark = pytest.mark.gpu
TOL_MEAN = 1e-9
TOL_VAR = 1e-8


@pytest.fixture(scope="module")
def argus():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2510_11077_amd as A
    return A


@pytest.fixture(params=["auto", "seq", "tp2", "tp4", "tp16"])
def form(request, monkeypatch):
    """Smoother form: the tuner's choice, the one-wave-per-item sweep, or the
    time-parallel form with the longest pulsar in 2, 4 or
    16 chunks (shorter pulsars in proportionally fewer, at most one per
    level-1 segment)."""
    if request.param == "auto":
        monkeypatch.delenv("ARGUS_SMOOTH", raising=False)
    else:
        monkeypatch.setenv("ARGUS_SMOOTH", request.param)
    return request.param


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build()
    return oracle


def dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def gpu_smooth(A, d, th, want_var=True):
    ds = A.Dataset(d)
    m, v, ll, st = ds.smooth(dev(th), want_var=want_var)
    # [N, nc, S] -> [S, N, nc]
    m = m.cpu().numpy().transpose(2, 0, 1)
    v = None if v is None else v.cpu().numpy().transpose(2, 0, 1)
    return m, v, ll.cpu().numpy(), st.cpu().numpy()


def check(m, v, rm, rv):
    nan = np.isnan(rm)
    assert np.array_equal(np.isnan(m), nan) and np.array_equal(np.isnan(v), np.isnan(rv))
    ok = ~nan
    m, v, rm, rv = m[ok], v[ok], rm[ok], rv[ok]
    zero = rv == 0.0
    assert np.array_equal(v[zero], rv[zero]) and np.array_equal(m[zero], rm[zero])
    pos = ~zero
    assert (rv[pos] > 0).all()
    em = np.abs(m[pos] - rm[pos]) / np.sqrt(rv[pos])
    ev = np.abs(v[pos] - rv[pos]) / rv[pos]
    assert em.max(initial=0.0) <= TOL_MEAN, em.max()
    assert ev.max(initial=0.0) <= TOL_VAR, ev.max()
    return em.max(initial=0.0), ev.max(initial=0.0)


def run(A, orc, d, th):
    m, v, ll, st = gpu_smooth(A, d, th)
    c = d.to_canon(th)
    rm, rv, rst = orc.smooth(d, c)
    assert np.array_equal(st, rst)
    check(m, v, rm, rv)
    ref_ll, _ = orc.loglike(d, c)
    ok = rst == 0
    assert np.array_equal(ll[~ok], ref_ll[~ok])
    assert (np.abs(ll[ok] - ref_ll[ok]) <= 1e-9 * np.maximum(np.abs(ref_ll[ok]), 1.0)).all()
    return m, v


def test_spin_model(argus, orc, form):
    d = pi.make_config("cfg1")
    run(argus, orc, d, pi.sample_theta(d, 64, pi.THETA_SEED["cfg1"]))


@pytest.mark.parametrize("S", [1, 63, 65, 130])
def test_pulsars_ragged_tiles(argus, orc, form, S):
    """Stream lengths 1 (smoothed = filtered), 0 (nothing written), around
    the 4-TOA reverse pieces and the level-1 segments, and sample counts
    around the 64-lane tile."""
    d = pi.make_pta("t", n_psr=6, counts=[1, 0, 37, 64, 130, 257], seed=31)
    run(argus, orc, d, pi.sample_theta(d, S, 7 + S))


def test_prior_corners(argus, orc, form):
    d = pi.make_pta("t", n_psr=3, counts=[2000, 1500, 200], seed=33)
    lo, hi = d.lo, d.hi
    rng = np.random.default_rng(5)
    th = [lo, hi, np.where(np.arange(lo.size) % 2, lo, hi), np.where(np.arange(lo.size) % 2, hi, lo)]
    th += [np.where(rng.random(lo.size) < 0.5, lo, hi) for _ in range(12)]
    run(argus, orc, d, np.array(th))
    d1 = pi.make_config("cfg1")
    run(argus, orc, d1, np.array([d1.lo, d1.hi, [d1.lo[0], d1.hi[1]], [d1.hi[0], d1.lo[1]]]))


def test_free_mask_subset(argus, orc):
    d = pi.make_config("cfg5")
    run(argus, orc, d, pi.sample_theta(d, 70, 56))


def test_failures_and_deterministic_states(argus, orc, form):
    d = pi.make_pta("t", n_psr=3, counts=[10, 12, 8], seed=34)
    th = np.tile(d.truth, (4, 1))
    th[1, 5] = np.nan   # pulsar 1's own parameter: only its entries are NaN
    th[2, -1] = np.inf  # common gamma: every pulsar
    th[3, 2] = 0.0      # EFAC 0 of pulsar 0 (EQUAD keeps S > 0)
    run(argus, orc, d, th)
    dz = pi.make_pta("t", n_psr=2, counts=[6, 7], seed=48)
    dz.s_r = dz.s_f = dz.sigma_s = 0.0
    z = np.tile(dz.truth, (2, 1))
    z[0, [0, 2, 3]] = [-400.0, 0.0, -400.0]
    z[0, -2] = -400.0   # pulsar 0: every variance zero -> NONPD, NaN
    m, v = run(argus, orc, dz, z)
    assert (m[1, :, :2] == 0).all() and (v[1, :, :2] == 0).all()


def test_means_only_and_repeatable(argus, orc, form):
    import torch
    d = pi.make_pta("t", n_psr=4, counts=[300, 7, 1200, 64], seed=36)
    th = dev(pi.sample_theta(d, 100, 8))
    ds = argus.Dataset(d)
    m1, v1, ll1, st1 = ds.smooth(th)
    m2, v2, ll2, _ = ds.smooth(th, want_var=False)
    assert v2 is None
    assert torch.equal(m1, m2) and torch.equal(ll1, ll2)
    m3, v3, _, _ = ds.smooth(th)
    assert torch.equal(m1, m3) and torch.equal(v1, v3)
    ll0, st0 = ds.loglike(th)
    assert torch.equal(st0, st1)
    assert (torch.abs(ll0 - ll1) <= 1e-9 * torch.clamp(torch.abs(ll0), min=1.0)).all()


def test_cfg4_full_batch_sampled(argus, orc, form):
    """47 pulsars (about 37k TOAs), 1024 samples, launched as the benchmark
    launches it; the oracle checks three samples over every TOA."""
    import torch
    d = pi.make_config("cfg4")
    th = pi.sample_theta(d, pi.N_SAMPLES["cfg4"], pi.THETA_SEED["cfg4"])
    ds = argus.Dataset(d)
    m, v, ll, st = ds.smooth(dev(th))
    assert bool((st == 0).all()) and bool(torch.isfinite(m).all()) and bool((v > 0).all())
    idx = [0, 511, 1023]
    m = m[:, :, idx].cpu().numpy().transpose(2, 0, 1)
    v = v[:, :, idx].cpu().numpy().transpose(2, 0, 1)
    rm, rv, rst = orc.smooth(d, d.to_canon(th[idx]))
    assert (rst == 0).all()
    check(m, v, rm, rv)


def test_joint_model_unsupported(argus):
    d = pi.make_pta("t", n_psr=2, counts=[5, 6], seed=35, model=pi.M_JOINT)
    ds = argus.Dataset(d)
    with pytest.raises(argus.ArgusError, match="models 1, 2 and 4"):
        ds.smooth(dev(pi.sample_theta(d, 2, 1)))


def test_spin_noise_after_a_long_gap(argus, orc, form):
    """About 800 days without TOAs under the strongest spin noise of the
    prior: the predicted residual variance then exceeds the white variance
    by about 13 decades, where a covariance update that subtracts u u^T / S
    with the rounded S would lose most digits of the filtered variance."""
    import dataclasses
    d = pi.make_spin("t1", n_toa=200, seed=9)
    keep = np.r_[0:25, 75:100]
    d = dataclasses.replace(d, t=d.t[keep], y=d.y[keep], sigma=d.sigma[keep],
                            off=np.array([0, keep.size], np.int64))
    th = np.array([[d.hi[0], 1.0], [d.hi[0] - 0.5, 0.9], [d.lo[0], 1.1]])
    run(argus, orc, d, th)


@pytest.mark.parametrize("S", [1, 70])
def test_dm_model_ragged_tiles(argus, orc, form, S):
    """Model 4 (state r, f, a, g, m; chromatic factor per TOA): empty,
    one-TOA and ragged pulsars, partial tiles."""
    d = pi.make_pta_dm("t", n_psr=6, counts=[1, 0, 37, 64, 130, 257], seed=61)
    th = pi.sample_theta(d, S, 62)
    m, v = run(argus, orc, d, th)
    assert m.shape[2] == 5


def test_dm_model_long_pulsar_near_truth(argus, orc, form):
    """Several checkpoint segments and 4-TOA pieces, and posteriors much
    tighter than the priors."""
    d = pi.make_pta_dm("t", n_psr=2, counts=[1500, 333], seed=63)
    th = pi.theta_near_truth(d, 64, 64, scale=0.05)
    run(argus, orc, d, th)


def test_dm_model_prior_corners(argus, orc, form):
    d = pi.make_pta_dm("t", n_psr=3, counts=[40, 25, 60], seed=65)
    lo, hi = d.lo[d.free], d.hi[d.free]
    rng = np.random.default_rng(66)
    th = np.where(rng.random((16, lo.size)) < 0.5, lo, hi)
    run(argus, orc, d, th)


def test_dm_full_batch_sampled(argus, orc, form):
    """47 pulsars with DM variations (about 37k TOAs), 1024 samples, launched
    as the benchmark launches it; the oracle checks three samples."""
    import torch
    d = pi.make_config("cfg2dm")
    th = pi.sample_theta(d, 1024, pi.THETA_SEED["cfg2dm"])
    ds = argus.Dataset(d)
    m, v, ll, st = ds.smooth(dev(th))
    assert bool((st == 0).all()) and bool(torch.isfinite(m).all()) and bool((v > 0).all())
    idx = [0, 511, 1023]
    m = m[:, :, idx].cpu().numpy().transpose(2, 0, 1)
    v = v[:, :, idx].cpu().numpy().transpose(2, 0, 1)
    rm, rv, rst = orc.smooth(d, d.to_canon(th[idx]))
    assert (rst == 0).all()
    check(m, v, rm, rv)


def test_dm_failures(argus, orc, form):
    """Model 4: a non-finite DM parameter of one pulsar makes only that
    pulsar's entries NaN; a non-finite common parameter makes all of them NaN;
    the status words follow the oracle's."""
    d = pi.make_pta_dm("t", n_psr=3, counts=[10, 12, 8], seed=67)
    col = np.cumsum(d.free) - 1          # canonical index -> theta column
    amp, rate = 6 * 1 + 4, 6 * 1 + 5     # pulsar 1's log10 sigma_dm, log10 gamma_dm
    assert d.free[amp] and d.free[rate] and d.free[-1]
    th = np.tile(d.truth, (4, 1))
    th[1, col[amp]] = np.nan
    th[2, col[rate]] = np.inf
    th[3, col[-1]] = np.nan
    m, v = run(argus, orc, d, th)
    n0, n1 = 10, 12
    assert np.isnan(m[1, n0:n0 + n1]).all() and not np.isnan(m[1, :n0]).any()
    assert np.isnan(m[3]).all()
