"""Parity of the HIP likelihood kernels with the CPU oracle, element by
element, through the C ABI. Tolerance: |logL_gpu - logL_oracle| <=
1e-9 max(|logL_oracle|, 1) (FP64 on both sides; the residual difference is
rounding order: structured vs dense Joseph update, log-product vs per-step
log, hardware reciprocal)."""
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


def check(gpu_ll, gpu_st, ref_ll, ref_st, tol=TOL):
    gpu_ll = gpu_ll.cpu().numpy() if hasattr(gpu_ll, "cpu") else gpu_ll
    gpu_st = gpu_st.cpu().numpy() if hasattr(gpu_st, "cpu") else gpu_st
    assert np.array_equal(gpu_st, ref_st), (gpu_st, ref_st)
    ok = ref_st == 0
    assert np.array_equal(gpu_ll[~ok], ref_ll[~ok])  # -inf where failed
    err = np.abs(gpu_ll[ok] - ref_ll[ok]) / np.maximum(np.abs(ref_ll[ok]), 1.0)
    assert err.max(initial=0.0) <= tol, err.max()
    return err.max(initial=0.0)


def run(A, orc, d, theta, plain=False):
    ds = A.Dataset(d)
    th = dev(theta)
    if plain:
        ll, st = ds.loglike_plain(th)
    else:
        ll, st = ds.loglike(th)
    ref, rst = orc.loglike(d, d.to_canon(theta))
    return check(ll, st, ref, rst)


def test_spin_model_cfg1(argus, orc):
    d = pi.make_config("cfg1")
    th = pi.sample_theta(d, 64, pi.THETA_SEED["cfg1"])
    run(argus, orc, d, th)


@pytest.mark.parametrize("S", [1, 63, 64, 65, 130])
def test_pulsars_ragged_tiles(argus, orc, S):
    d = pi.make_pta("t", n_psr=6, counts=[1, 0, 37, 64, 130, 257], seed=31)
    th = pi.sample_theta(d, S, 7 + S)
    run(argus, orc, d, th)


def test_per_pulsar_terms(argus, orc):
    d = pi.make_pta("t", n_psr=5, counts=[3, 90, 0, 200, 17], seed=32)
    th = pi.sample_theta(d, 70, 3)
    ds = argus.Dataset(d)
    terms, st = ds.loglike_terms(dev(th))
    ref, rst, per = orc.loglike(d, d.to_canon(th), per_psr=True)
    assert (st.cpu().numpy() == 0).all() and (rst == 0).all()
    t = terms.cpu().numpy().T
    err = np.abs(t - per) / np.maximum(np.abs(per), 1.0)
    assert err.max() <= TOL
    assert (t[:, 2] == 0.0).all()  # empty pulsar contributes exactly 0


def test_cfg2_full_batch(argus, orc):
    """47 pulsars, 4096 samples, launched exactly as the benchmark launches
    it (autotuned persistent kernel replayed from a graph)."""
    d = pi.make_config("cfg2")
    th = pi.sample_theta(d, pi.N_SAMPLES["cfg2"], pi.THETA_SEED["cfg2"])
    ds = argus.Dataset(d)
    t = dev(th)
    ll, st = ds.loglike(t)
    ll2, st2 = ds.loglike(t)  # graph replay
    ref, rst = orc.loglike(d, d.to_canon(th))
    check(ll, st, ref, rst)
    assert np.array_equal(ll.cpu().numpy(), ll2.cpu().numpy())


@pytest.mark.parametrize("cfg", ["cfg1", "cfg2"])
def test_plain_baseline(argus, orc, cfg):
    d = pi.make_config(cfg)
    th = pi.sample_theta(d, 8, 99)
    run(argus, orc, d, th, plain=True)


def test_prior_corners(argus, orc):
    d = pi.make_pta("t", n_psr=4, counts=[150, 20, 300, 80], seed=33)
    lo, hi = d.lo, d.hi
    rng = np.random.default_rng(5)
    corners = [lo, hi, np.where(np.arange(lo.size) % 2, lo, hi), np.where(np.arange(lo.size) % 2, hi, lo)]
    corners += [np.where(rng.random(lo.size) < 0.5, lo, hi) for _ in range(60)]
    run(argus, orc, d, np.array(corners))
    d1 = pi.make_config("cfg1")
    run(argus, orc, d1, np.array([d1.lo, d1.hi, [d1.lo[0], d1.hi[1]], [d1.hi[0], d1.lo[1]]]))


def test_status_flags(argus, orc):
    d = pi.make_pta("t", n_psr=3, counts=[10, 12, 8], seed=34)
    th = np.tile(d.truth, (6, 1))
    th[1, 2] = np.nan            # EFAC of pulsar 0
    th[2, 9] = np.inf            # log10 gamma of pulsar 2
    th[3, -1] = np.nan           # common gamma
    th[4, 5] = np.nan            # pulsar 1
    run(argus, orc, d, th)
    dz = pi.make_pta("t", n_psr=3, counts=[10, 12, 8], seed=34)
    dz.s_r = dz.s_f = dz.sigma_s = 0.0
    z = np.tile(d.truth, (3, 1))
    z[0, [0, 4, 8]] = -400.0
    z[0, [2, 6, 10]] = 0.0
    z[0, [3, 7, 11]] = -400.0
    z[0, -2] = -400.0            # sample 0: every variance is exactly zero -> NONPD
    z[1, 2] = 0.0                # sample 1: EFAC 0 alone keeps S > 0
    ds = argus.Dataset(dz)
    ll, st = ds.loglike(dev(z))
    ref, rst = orc.loglike(dz, z)
    assert rst[0] == 1
    check(ll, st, ref, rst)


def test_fast_form_hands_items_over_exactly(argus, orc):
    """The batched 4-state filter runs a fast loop that leaves to the general
    loop every (64-sample tile, pulsar) item in which some innovation
    variance falls below 2^-120, a parameter is not finite, or the red-noise
    rate times the pulsar's longest interval is too large for its expm1.
    Here TOA errors of ~1e-25 s, no spin terms, and, in every third of the
    first 128 samples, EQUAD, red and common amplitudes of 1e-40 keep S near
    1e-50 in those samples, so some tiles mix handed-over and fast lanes and
    others are fast throughout; a few samples carry huge rates. Every sample
    matches the oracle."""
    d = pi.make_pta("t", n_psr=3, counts=[300, 70, 129], seed=41)
    d.sigma = d.sigma * 1e-18
    d.s_r = d.s_f = d.sigma_s = 0.0
    th = pi.sample_theta(d, 200, 42)
    tiny = (np.arange(200) % 3 == 0) & (np.arange(200) < 128)
    for p in range(3):
        th[tiny, 4 * p] = -40.0      # log10 sigma_red
        th[tiny, 4 * p + 3] = -40.0  # log10 EQUAD
    th[tiny, -2] = -40.0             # log10 A
    th[150:153, 1] = 4.0             # log10 gamma_red of pulsar 0: rate 1e4 / s
    err = run(argus, orc, d, th)
    print("max rel err %.2e" % err)


def test_empty_batch_is_a_noop(argus):
    import torch
    d = pi.make_pta("t", n_psr=2, counts=[5, 6], seed=35)
    ds = argus.Dataset(d)
    out = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    ds.loglike(torch.empty((0, ds.n_params), dtype=torch.float64, device="cuda"), out=out[:0])
    assert out.item() == 7.0


def test_repeatable_and_graph_replays(argus, orc):
    """Bitwise repeatable (no float atomics), across graph replays with
    eager work in between and after re-capture for new output buffers."""
    import torch
    d = pi.make_pta("t", n_psr=8, counts=[40, 300, 7, 120, 2000, 1, 60, 500], seed=36)
    th = pi.sample_theta(d, 300, 8)
    ds = argus.Dataset(d)
    t = dev(th)
    first, st = ds.loglike(t)
    first = first.clone()
    for i in range(4):
        junk = torch.randn(1 << 20, device="cuda").sum()
        out = torch.empty(300, dtype=torch.float64, device="cuda")
        ll, _ = ds.loglike(t, out=out if i % 2 else None)
        torch.cuda.synchronize()
        assert torch.equal(ll, first)
        del junk
    ref, rst = orc.loglike(d, d.to_canon(th))
    check(first, st, ref, rst)


def test_free_mask_subset(argus, orc):
    d = pi.make_config("cfg5")
    th = pi.sample_theta(d, 100, 55)
    assert th.shape[1] == 10
    run(argus, orc, d, th)


# ------------------------------------------------------------ joint model
@pytest.fixture(params=["blocked", "seq"])
def joint_form(request, monkeypatch):
    """The joint model's kernel: the blocked one (the default up to 22
    pulsars) or the sequential one (the default above), forced through
    ARGUS_JOINT=seq."""
    if request.param == "seq":
        monkeypatch.setenv("ARGUS_JOINT", "seq")
    else:
        monkeypatch.delenv("ARGUS_JOINT", raising=False)
    return request.param


def test_joint_small(argus, orc, joint_form):
    d = pi.make_pta("t", n_psr=3, counts=[30, 1, 45], seed=37, model=pi.M_JOINT)
    th = pi.sample_theta(d, 6, 9)
    run(argus, orc, d, th)


def test_joint_tied_toas(argus, orc, joint_form):
    d = pi.make_pta("t", n_psr=2, counts=[15, 15], seed=38, model=pi.M_JOINT)
    d.t[15:] = d.t[:15]
    run(argus, orc, d, pi.sample_theta(d, 4, 10))


def test_joint_twenty_pulsars(argus, orc, joint_form):
    d = pi.make_pta("t", n_psr=20, counts=np.full(20, 40), seed=39, model=pi.M_JOINT)
    th = pi.sample_theta(d, 6, 11)
    run(argus, orc, d, th)


def test_joint_cfg3_sampled(argus, orc):
    """Full cfg3 (20 pulsars x 1000 TOAs, 256 samples) at the benchmark's
    launch; the oracle (dense 80 x 80 Joseph form) checks two samples."""
    d = pi.make_config("cfg3")
    th = pi.sample_theta(d, pi.N_SAMPLES["cfg3"], pi.THETA_SEED["cfg3"])
    ds = argus.Dataset(d)
    ll, st = ds.loglike(dev(th))
    idx = [0, 255]
    ref, rst = orc.loglike(d, d.to_canon(th[idx]))
    check(ll.cpu().numpy()[idx], st.cpu().numpy()[idx], ref, rst)
    assert (st.cpu().numpy() == 0).all()
    assert np.isfinite(ll.cpu().numpy()).all()


def test_joint_cfg3_blocked_against_sequential(argus, monkeypatch):
    """Full cfg3 (20 pulsars x 1000 TOAs, 256 samples): the blocked kernel
    (16-TOA elimination, MFMA downdate) against the sequential kernel (one
    TOA at a time; its own parity with the oracle is tested above) on every
    sample. The two are different fp64 algebra for the same recursion; the
    bound is the oracle tolerance of this module."""
    import torch
    d = pi.make_config("cfg3")
    th = dev(pi.sample_theta(d, pi.N_SAMPLES["cfg3"], pi.THETA_SEED["cfg3"]))
    ds = argus.Dataset(d)
    monkeypatch.delenv("ARGUS_JOINT", raising=False)
    ll_b, st_b = ds.loglike(th)
    ll_b, st_b = ll_b.clone(), st_b.clone()
    monkeypatch.setenv("ARGUS_JOINT", "seq")
    ll_s, st_s = ds.loglike(th)
    assert torch.equal(st_b, st_s) and bool((st_b == 0).all())
    check(ll_b.cpu().numpy(), st_b.cpu().numpy(), ll_s.cpu().numpy(), st_s.cpu().numpy())


@pytest.mark.parametrize("counts", [[1], [9, 8], [5, 0, 12], [3] * 22])
def test_joint_block_edges(argus, orc, counts, joint_form):
    """Stream lengths around the 16-TOA block size, an empty pulsar, and the
    largest supported joint model (22 pulsars, padded MFMA tiles)."""
    d = pi.make_pta("t", n_psr=len(counts), counts=counts, seed=40 + len(counts),
                    model=pi.M_JOINT)
    run(argus, orc, d, pi.sample_theta(d, 5, 12))


def test_joint_prior_corners_and_flags(argus, orc, joint_form):
    d = pi.make_pta("t", n_psr=4, counts=[20, 35, 3, 50], seed=47, model=pi.M_JOINT)
    lo, hi = d.lo, d.hi
    th = np.array([lo, hi, np.where(np.arange(lo.size) % 2, lo, hi), d.truth, d.truth])
    th[3, 5] = np.nan
    th[4, -1] = np.inf
    run(argus, orc, d, th)
    dz = pi.make_pta("t", n_psr=2, counts=[6, 7], seed=48, model=pi.M_JOINT)
    dz.s_r = dz.s_f = dz.sigma_s = 0.0
    z = np.tile(dz.truth, (2, 1))
    z[0, [0, 4]] = -400.0
    z[0, [2, 6]] = 0.0
    z[0, [3, 7]] = -400.0
    z[0, -2] = -400.0
    ds = argus.Dataset(dz)
    ll, st = ds.loglike(dev(z))
    ref, rst = orc.loglike(dz, z)
    assert rst[0] == 1
    check(ll, st, ref, rst)


@pytest.mark.parametrize("P, per", [(23, 4), (45, 3), (55, 3), (63, 2)])
def test_joint_beyond_blocked_limit(argus, orc, P, per):
    """Arrays larger than the blocked kernel's LDS layout take the sequential
    kernel: one covariance block per thread up to 44 pulsars (23), two (45),
    four (55, and 63, the largest supported array); ragged TOA counts, and
    the oracle's dense 4P-state Joseph-form filter on every sample."""
    counts = np.full(P, per)
    counts[::3] += 1
    counts[1::5] = 1
    d = pi.make_pta("t", n_psr=P, counts=counts, seed=60 + P, model=pi.M_JOINT)
    run(argus, orc, d, pi.sample_theta(d, 3, 13 + P))


@pytest.mark.parametrize("cfg", ["64,7,0", "256,3,0", "1024,1,0,1", "256,1,0,1", "64,1,0,1",
                                 "64,5,1", "256,4,0,2", "512,3,0,2", "1024,1,0,2"])
def test_forced_launch_layouts(argus, orc, cfg, monkeypatch):
    """Every launch layout the tuner can pick gives the same parity: static
    longest-first with a grid smaller than the item count, one block per CU
    with per-SIMD lists (most lists here are empty; with one wave per block
    every list is drained by taking from the others), the global dynamic
    queue, and the time-parallel filter with 4, 8 and 16 chunks per item
    (fewer workgroups than items, streams shorter than the chunk count)."""
    monkeypatch.setenv("ARGUS_CFG", cfg)
    d = pi.make_pta("t", n_psr=7, counts=[400, 3, 0, 1200, 64, 777, 90], seed=49)
    th = pi.sample_theta(d, 200, 14)
    run(argus, orc, d, th)


# ------------------------------------------------ time-parallel filter
@pytest.mark.parametrize("nw", [4, 8, 16])
def test_time_parallel_spin_model(argus, orc, nw, monkeypatch):
    """The single-pulsar spin workload (500 TOAs, 64 samples) and its prior
    corners through the chunked scan, and the 800-day-gap stream where the
    predicted residual variance exceeds the white one by 13 decades."""
    import dataclasses
    monkeypatch.setenv("ARGUS_CFG", "%d,1,0,2" % (64 * nw))
    d = pi.make_config("cfg1")
    run(argus, orc, d, pi.sample_theta(d, 64, pi.THETA_SEED["cfg1"]))
    run(argus, orc, d, np.array([d.lo, d.hi, [d.lo[0], d.hi[1]], [d.hi[0], d.lo[1]]]))
    g = pi.make_spin("t1", n_toa=200, seed=9)
    keep = np.r_[0:25, 75:100]
    g = dataclasses.replace(g, t=g.t[keep], y=g.y[keep], sigma=g.sigma[keep],
                            off=np.array([0, keep.size], np.int64))
    run(argus, orc, g, np.array([[g.hi[0], 1.0], [g.hi[0] - 0.5, 0.9], [g.lo[0], 1.1]]))


@pytest.mark.parametrize("nw", [4, 8, 16])
def test_time_parallel_per_pulsar_model(argus, orc, nw, monkeypatch):
    monkeypatch.setenv("ARGUS_CFG", "%d,2,0,2" % (64 * nw))
    d = pi.make_pta("t", n_psr=5, counts=[2000, 3, 0, 17, 600], seed=50)
    lo, hi = d.lo, d.hi
    th = np.vstack([pi.sample_theta(d, 60, 15), [lo, hi, np.where(np.arange(lo.size) % 2, lo, hi)]])
    run(argus, orc, d, th)


def test_time_parallel_status_flags(argus, orc, monkeypatch):
    monkeypatch.setenv("ARGUS_CFG", "512,1,0,2")
    test_status_flags(argus, orc)


def test_time_parallel_is_chosen_for_one_item(argus):
    """With one (tile, pulsar) item the tuner times the chunked scan against
    the sequential layouts; the report names what it chose."""
    import torch
    d = pi.make_config("cfg1")
    ds = argus.Dataset(d)
    ds.loglike(dev(pi.sample_theta(d, 64, 1)))
    torch.cuda.synchronize()
    info = ds.tune_info(64)
    assert "order=2" in info
