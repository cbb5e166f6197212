"""Gradient of the batched likelihood against the oracle's complex-step
derivative and against central differences of the GPU likelihood, for both
gradient sweeps (every test runs with the tangent sweep, the default, and
with the reverse-mode adjoint). Tolerances: ||g - g_ref||_inf <= 1e-9 max(||g_ref||_inf, 1) per
sample row and, per component, |g_j - g_ref,j| <= 1e-9 (|g_ref,j| +
1e-3 ||g_ref||_inf); central differences (h = 1e-6): 1e-5 max(|g_j|, 1)."""
import numpy as np
import pytest

import pta_inputs as pi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def argus():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2510_11077_amd as A
    return A


@pytest.fixture(autouse=True, params=["tangent", "adjoint"])
def sweep(request, monkeypatch):
    if request.param == "adjoint":
        monkeypatch.setenv("ARGUS_GRAD", "adjoint")
    else:
        monkeypatch.delenv("ARGUS_GRAD", raising=False)
    return request.param


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build()
    return oracle


def dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def check_grad(g, gref, tol=1e-9):
    g = np.asarray(g)
    for s in range(gref.shape[0]):
        inf = np.abs(gref[s]).max()
        d = np.abs(g[s] - gref[s])
        assert d.max() <= tol * max(inf, 1.0), (s, d.max(), inf)
        assert (d <= tol * (np.abs(gref[s]) + 1e-3 * inf)).all(), (s, np.argmax(d / (np.abs(gref[s]) + 1e-3 * inf)))


def oracle_grad(orc, d, th):
    """Complex-step d logL / d theta (free columns only)."""
    return orc.grad_cs(d, d.to_canon(th), which=d.free_idx)


def test_grad_ragged_pulsars(argus, orc):
    d = pi.make_pta("t", n_psr=5, counts=[1, 0, 7, 37, 130], seed=41)
    th = pi.sample_theta(d, 70, 3)
    ds = argus.Dataset(d)
    ll, g, st = ds.loglike_grad(dev(th))
    assert (st.cpu().numpy() == 0).all()
    check_grad(g.cpu().numpy(), oracle_grad(orc, d, th))
    ref, _ = orc.loglike(d, d.to_canon(th))
    assert (np.abs(ll.cpu().numpy() - ref) <= 1e-9 * np.maximum(np.abs(ref), 1)).all()


def test_grad_long_pulsar_segments(argus, orc):
    """N_p = 2000 exercises many level-1 segments and level-2 pieces."""
    d = pi.make_pta("t", n_psr=2, counts=[2000, 333], seed=42)
    th = pi.sample_theta(d, 64, 4)
    ds = argus.Dataset(d)
    _, g, _ = ds.loglike_grad(dev(th))
    check_grad(g.cpu().numpy(), oracle_grad(orc, d, th))


def test_grad_spin_model(argus, orc):
    d = pi.make_config("cfg1")
    th = pi.sample_theta(d, 64, 5)
    ds = argus.Dataset(d)
    _, g, _ = ds.loglike_grad(dev(th))
    check_grad(g.cpu().numpy(), oracle_grad(orc, d, th))


def test_grad_cfg4_sampled(argus, orc):
    """47 pulsars, 1024 samples; the oracle checks 16 rows."""
    d = pi.make_config("cfg4")
    th = pi.sample_theta(d, pi.N_SAMPLES["cfg4"], pi.THETA_SEED["cfg4"])
    ds = argus.Dataset(d)
    ll, g, st = ds.loglike_grad(dev(th))
    assert (st.cpu().numpy() == 0).all()
    rows = np.arange(0, 1024, 64)
    check_grad(g.cpu().numpy()[rows], oracle_grad(orc, d, th[rows]))
    # the likelihood of the gradient call is the likelihood
    l2, _ = ds.loglike(dev(th))
    assert np.allclose(ll.cpu().numpy(), l2.cpu().numpy(), rtol=1e-12, atol=0)


def test_grad_vs_central_differences(argus):
    d = pi.make_pta("t", n_psr=3, counts=[200, 50, 120], seed=43)
    th = pi.sample_theta(d, 8, 6)
    ds = argus.Dataset(d)
    _, g, _ = ds.loglike_grad(dev(th))
    g = g.cpu().numpy()
    h = 1e-6
    for j in range(th.shape[1]):
        tp, tm = th.copy(), th.copy()
        tp[:, j] += h
        tm[:, j] -= h
        fp, _ = ds.loglike(dev(tp))
        fm, _ = ds.loglike(dev(tm))
        fd = (fp.cpu().numpy() - fm.cpu().numpy()) / (2 * h)
        assert (np.abs(fd - g[:, j]) <= 1e-5 * np.maximum(np.abs(g[:, j]), 1.0)).all(), j


def test_grad_free_mask_columns(argus, orc):
    d = pi.make_config("cfg5")
    th = pi.sample_theta(d, 50, 7)
    ds = argus.Dataset(d)
    _, g, _ = ds.loglike_grad(dev(th))
    assert g.shape == (50, 10)
    check_grad(g.cpu().numpy(), oracle_grad(orc, d, th))


def test_grad_failed_rows_are_zero(argus, orc):
    d = pi.make_pta("t", n_psr=2, counts=[20, 30], seed=44)
    th = np.tile(d.truth, (3, 1))
    th[1, 5] = np.nan
    ds = argus.Dataset(d)
    ll, g, st = ds.loglike_grad(dev(th))
    st, g, ll = st.cpu().numpy(), g.cpu().numpy(), ll.cpu().numpy()
    assert st[1] == 2 and ll[1] == -np.inf and not g[1].any()
    assert st[0] == 0 and np.isfinite(g[0]).all()
    check_grad(g[[0, 2]], oracle_grad(orc, d, th[[0, 2]]))


def test_autograd_function(argus):
    import torch
    d = pi.make_pta("t", n_psr=3, counts=[40, 60, 25], seed=45)
    th = dev(pi.sample_theta(d, 16, 8)).requires_grad_(True)
    ds = argus.Dataset(d)
    w = torch.linspace(0.5, 2.0, 16, dtype=torch.float64, device="cuda")
    out = argus.ArgusLogLike.apply(th, ds)
    (out * w).sum().backward()
    _, g, _ = ds.loglike_grad(th.detach())
    assert torch.allclose(th.grad, g * w[:, None], rtol=0, atol=0)


def test_grad_repeatable(argus):
    d = pi.make_pta("t", n_psr=4, counts=[300, 10, 90, 1], seed=46)
    th = dev(pi.sample_theta(d, 130, 9))
    ds = argus.Dataset(d)
    _, g1, _ = ds.loglike_grad(th)
    g1 = g1.clone()
    _, g2, _ = ds.loglike_grad(th)
    assert np.array_equal(g1.cpu().numpy(), g2.cpu().numpy())


@pytest.mark.parametrize("nd", ["1", "2", "3", "6", "1,2,90", "1,3,90", "2,3,3", "1,3,261", "pc", "pc1"])
def test_tangent_direction_splits(argus, orc, nd, sweep, monkeypatch):
    """The tangent sweep with each split of the six directions over waves:
    uniform, and mixed (fewer directions per wave for pulsars of at least the
    threshold's TOAs; "1,3,261" puts every pulsar in the second group); "pc"
    and "pc1" are the producer/consumer forms (the base filter on one wave,
    its per-TOA values handed through LDS to three waves (the red rate alone,
    two pairs of directions; the common variance's tangent gives both log10 A
    and gamma) or five of one), here with a pulsar of no TOAs and one of fewer
    TOAs than a hand-over block."""
    if sweep != "tangent":
        pytest.skip("tangent sweep only")
    monkeypatch.setenv("ARGUS_TAN_ND", nd)
    d = pi.make_pta("t", n_psr=4, counts=[90, 3, 0, 260], seed=51)
    th = pi.sample_theta(d, 66, 17)
    ll, g, st = argus.Dataset(d).loglike_grad(dev(th))
    assert (st.cpu().numpy() == 0).all()
    check_grad(g.cpu().numpy(), oracle_grad(orc, d, th))
