"""argus_loglike_noalloc (the batched likelihood for callers that cannot
allocate device memory) against argus_loglike on the same inputs, through
the C ABI: two calls in a row on one dataset, the second with fewer
samples, for models 2, 1 and 4; failures flagged alike; an S beyond the
static scratch is rejected on the host. Both entry points run the same
filter and reduction kernels, so the bar is the likelihood's 1e-9 relative
(equality is expected)."""
import numpy as np
import pytest

import pta_inputs as pi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2510_11077_amd as A
    return A


def dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def compare(A, ds, th):
    import torch
    S = th.shape[0]
    ref, rst = ds.loglike(th)
    out = torch.empty(S, dtype=torch.float64, device="cuda")
    st = torch.empty(S, dtype=torch.int32, device="cuda")
    got, gst = ds.loglike_noalloc(th, out, st)
    torch.cuda.synchronize()
    r, g = ref.cpu().numpy(), got.cpu().numpy()
    assert np.array_equal(gst.cpu().numpy(), rst.cpu().numpy())
    fin = np.isfinite(r)
    assert np.array_equal(fin, np.isfinite(g))
    err = np.abs(g[fin] - r[fin]) / np.maximum(np.abs(r[fin]), 1.0)
    assert err.size == 0 or err.max() <= 1e-9, err.max()
    return r, g


@pytest.mark.parametrize("cfg,sizes", [("cfg2", (4096, 1000)), ("cfg1", (64, 7)),
                                       ("cfg2dm", (1000, 65))])
def test_noalloc_matches_loglike(A, cfg, sizes):
    d = pi.make_config(cfg)
    ds = A.Dataset(d)
    th = pi.sample_theta(d, max(sizes), pi.THETA_SEED[cfg])
    for S in sizes:  # the second call is smaller and reuses the same scratch
        print("no-alloc likelihood: %s, S=%d" % (cfg, S), flush=True)
        compare(A, ds, dev(th[:S]))


def test_noalloc_failures_and_limit(A):
    import torch
    d = pi.make_pta("t", n_psr=3, counts=[50, 0, 20], seed=5)
    ds = A.Dataset(d)
    th = pi.sample_theta(d, 130, 6)
    th[3, 0] = np.nan
    th[70, -1] = np.inf
    r, g = compare(A, ds, dev(th))
    assert np.isneginf(g[3]) and np.isneginf(g[70])
    # beyond the static scratch: rejected on the host, before any launch
    big = torch.zeros((800000, ds.n_params), dtype=torch.float64, device="cuda")
    with pytest.raises(A.ArgusError, match="no-allocation scratch"):
        ds.loglike_noalloc(big)
