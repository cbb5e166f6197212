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


def test_dm_unsupported_calls(argus):
    d = pi.make_pta_dm("t", n_psr=2, counts=[5, 6], seed=55)
    ds = argus.Dataset(d)
    th = dev(pi.sample_theta(d, 2, 1))
    with pytest.raises(argus.ArgusError, match="gradient"):
        ds.loglike_grad(th)
    with pytest.raises(argus.ArgusError, match="smoother"):
        ds.smooth(th)
