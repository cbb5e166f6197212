"""Parity of the model with DM variations (model 4: state [r, f, a, g, m],
chromatic factor (1400 / nu)^2 per TOA) on the GPU with the oracle, element
by element, through the C ABI. Tolerance as for the other likelihoods:
|logL_gpu - logL_oracle| <= 1e-9 max(|logL_oracle|, 1)."""
import numpy as np
import pytest

import pta_inputs as pi

pytestmark = pytest.mark.gpu
TOL = 1e-9


@pytest.fixture(scope="module")
def argus():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2510_11077_amd as A
    return A


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build()
    return oracle


def dev(x, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype or torch.float64, device="cuda")


def run(A, orc, d, th):
    ds = A.Dataset(d)
    ll, st = ds.loglike(dev(th))
    ref, rst = orc.loglike(d, d.to_canon(th))
    ll, st = ll.cpu().numpy(), st.cpu().numpy()
    assert np.array_equal(st, rst)
    ok = rst == 0
    assert np.array_equal(ll[~ok], ref[~ok])
    err = np.abs(ll[ok] - ref[ok]) / np.maximum(np.abs(ref[ok]), 1.0)
    assert err.max(initial=0.0) <= TOL, err.max()
    return ds


@pytest.mark.parametrize("S", [1, 65, 130])
def test_dm_ragged_tiles(argus, orc, S):
    d = pi.make_pta_dm("t", n_psr=6, counts=[1, 0, 37, 64, 130, 257], seed=51)
    run(argus, orc, d, pi.sample_theta(d, S, 60 + S))


def test_dm_terms_and_corners(argus, orc):
    d = pi.make_pta_dm("t", n_psr=4, counts=[150, 20, 300, 80], seed=52)
    lo, hi = d.lo, d.hi
    rng = np.random.default_rng(6)
    th = np.array([lo, hi, np.where(np.arange(lo.size) % 2, lo, hi)]
                  + [np.where(rng.random(lo.size) < 0.5, lo, hi) for _ in range(40)])
    ds = run(argus, orc, d, th)
    terms, st = ds.loglike_terms(dev(th))
    ref, rst, per = orc.loglike(d, d.to_canon(th), per_psr=True)
    t = terms.cpu().numpy().T
    assert (np.abs(t - per) / np.maximum(np.abs(per), 1.0)).max() <= TOL


def test_dm_status_flags(argus, orc):
    d = pi.make_pta_dm("t", n_psr=3, counts=[10, 12, 8], seed=53)
    th = np.tile(d.truth, (5, 1))
    th[1, 4] = np.nan        # log10 sigma_dm of pulsar 0
    th[2, 11] = np.inf       # log10 gamma_dm of pulsar 1
    th[3, -1] = np.nan       # common gamma
    th[4, 2] = 0.0           # EFAC 0 (EQUAD keeps S > 0)
    run(argus, orc, d, th)


def test_dm_full_batch(argus, orc):
    """47 pulsars observed in four bands, 4096 samples, the benchmark's
    launch (autotuned, graph replay); every sample against the oracle."""
    d = pi.make_config("cfg2dm")
    th = pi.sample_theta(d, pi.N_SAMPLES["cfg2dm"], pi.THETA_SEED["cfg2dm"])
    ds = run(argus, orc, d, th)
    ll2, _ = ds.loglike(dev(th))
    ll1, _ = ds.loglike(dev(th))
    import torch
    assert torch.equal(ll1, ll2)


@pytest.mark.parametrize("cfg", ["64,7,0", "1024,1,0,1", "64,5,1"])
def test_dm_forced_layouts(argus, orc, cfg, monkeypatch):
    monkeypatch.setenv("ARGUS_CFG", cfg)
    d = pi.make_pta_dm("t", n_psr=7, counts=[400, 3, 0, 1200, 64, 777, 90], seed=54)
    run(argus, orc, d, pi.sample_theta(d, 200, 15))


# ------------------------------------------------------------------ gradient
def check_grad(g, gref, tol=1e-9):
    """As for the other models: ||g - g_ref||_inf <= tol max(||g_ref||_inf, 1)
    per row and, per component, tol (|g_ref,j| + 1e-3 ||g_ref||_inf)."""
    for s in range(gref.shape[0]):
        inf = np.abs(gref[s]).max()
        d = np.abs(g[s] - gref[s])
        assert d.max() <= tol * max(inf, 1.0), (s, d.max(), inf)
        assert (d <= tol * (np.abs(gref[s]) + 1e-3 * inf)).all(), s


@pytest.mark.parametrize("nd", ["", "1", "2", "4", "1,2,37", "1,4,37", "2,4,7", "pc", "pc1"])
def test_dm_gradient(argus, orc, nd, monkeypatch):
    """The model-4 tangent sweep (eight directions per pulsar, split over
    8 / nd waves; "a,b,t": a per wave for pulsars of at least t TOAs, b for
    the others; "pc" / "pc1": the base filter on one wave handing its
    per-TOA values to four waves (three of two directions, one of the common
    variance, whose tangent gives both log10 A and gamma) or seven of one;
    "" lets the first call choose) against the oracle's complex-step
    derivative, ragged pulsars and tiles."""
    if nd:
        monkeypatch.setenv("ARGUS_TAN_ND", nd)
    else:
        monkeypatch.delenv("ARGUS_TAN_ND", raising=False)
    d = pi.make_pta_dm("t", n_psr=5, counts=[1, 0, 7, 37, 130], seed=56)
    th = pi.sample_theta(d, 70, 16)
    ds = argus.Dataset(d)
    ll, g, st = ds.loglike_grad(dev(th))
    assert (st.cpu().numpy() == 0).all()
    gref = orc.grad_cs(d, d.to_canon(th), which=d.free_idx)
    check_grad(g.cpu().numpy(), gref)
    ref, _ = orc.loglike(d, d.to_canon(th))
    assert (np.abs(ll.cpu().numpy() - ref) <= TOL * np.maximum(np.abs(ref), 1)).all()


def test_dm_gradient_full_data_sampled(argus, orc, monkeypatch):
    """The DM gradient on all 47 pulsars (37,269 TOAs in four bands) at 1024
    samples, the gradient benchmark's batch, in the launch the first call
    tunes (the producer/consumer form there); the oracle's complex-step
    derivative checks 8 rows spread over the batch."""
    monkeypatch.delenv("ARGUS_TAN_ND", raising=False)
    d = pi.make_config("cfg2dm")
    th = pi.sample_theta(d, 1024, pi.THETA_SEED["cfg2dm"])
    ds = argus.Dataset(d)
    ll, g, st = ds.loglike_grad(dev(th))
    assert (st.cpu().numpy() == 0).all()
    rows = np.arange(0, 1024, 128)
    check_grad(g.cpu().numpy()[rows], orc.grad_cs(d, d.to_canon(th[rows]), which=d.free_idx))
    ref, _ = orc.loglike(d, d.to_canon(th[rows]))
    got = ll.cpu().numpy()[rows]
    assert (np.abs(got - ref) <= TOL * np.maximum(np.abs(ref), 1)).all()


def test_dm_gradient_long_pulsar_and_free_mask(argus, orc):
    d = pi.make_pta_dm("t", n_psr=2, counts=[2000, 333], seed=57)
    d.free = np.zeros(d.truth.size, bool)
    d.free[[0, 1, 4, 5, 8, 10, 11, 12, 13]] = True
    th = pi.sample_theta(d, 64, 17)
    ds = argus.Dataset(d)
    _, g, _ = ds.loglike_grad(dev(th))
    check_grad(g.cpu().numpy(), orc.grad_cs(d, d.to_canon(th), which=d.free_idx))


def test_dm_hmc_transition(argus, orc):
    """One HMC transition of the DM model against the oracle transition on
    the same draws (the sampler sees model 4 through the gradient)."""
    import torch
    from oracle import hmc
    d = pi.make_pta_dm("t", n_psr=2, counts=[40, 25], seed=58)
    S, L = 16, 3
    th0 = pi.theta_near_truth(d, S, 18, scale=0.02)
    width = d.hi - d.lo
    inv_mass = (0.01 * width) ** 2
    rng = np.random.default_rng(19)
    z = rng.normal(size=th0.shape)
    logu = np.log(rng.random(S))
    ds = argus.Dataset(d)
    t = dev(th0)
    ll, g, _ = ds.loglike_grad(t)
    acc = torch.zeros(S, dtype=torch.int32, device="cuda")
    dh = torch.empty(S, dtype=torch.float64, device="cuda")
    ds.hmc_step(t, ll, g, dev(np.full(S, 0.2)), dev(inv_mass), dev(d.lo), dev(d.hi), dev(z),
                dev(logu), L, acc, dh)
    f = hmc.oracle_target(d, orc)
    l0, g0 = f(th0)
    rt, rl, _, racc, rdh = hmc.transition(th0, l0, g0, np.full(S, 0.2), inv_mass, d.lo, d.hi,
                                          z, logu, L, f)
    clear = np.abs(logu + rdh) > 1e-5
    assert np.array_equal(acc.cpu().numpy().astype(bool)[clear], racc[clear])
    fin = np.isfinite(rdh)
    assert (np.abs(dh.cpu().numpy()[fin] - rdh[fin]) <= 1e-6 + 1e-9 * np.abs(l0[fin])).all()
    a = racc & clear
    disp = np.max(np.abs(rt[a] - th0[a]), axis=1, keepdims=True)
    assert (np.abs(t.cpu().numpy()[a] - rt[a]) <= 1e-7 * disp).all()
