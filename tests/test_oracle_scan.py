"""Pins of the oracle's parallel-in-time filter (the Kalman recursion as an
associative scan over per-step elements, Sarkka & Garcia-Fernandez 2021)
against the sequential filter it must reproduce, in three evaluation orders
of the scan (left fold, recursive doubling, chunked): agreement of all three
with the sequential Joseph-form filter is what associativity and the
element definitions promise. CPU only.

Tolerances: the element algebra solves with I + C_i J_j, whose conditioning
grows with the information an element carries, so the scan keeps fewer
digits than the Joseph-form filter; the worst case measured on these inputs
(recursive doubling at prior corners of 4-state pulsars): log-likelihood
3.5e-10 relative, filtered means 8.3e-8 and covariances 5.5e-9 in units of
the filtered standard deviations. The bounds (3e-9, 1e-6) keep a 10x margin;
a wrong sign, index or operand order gives O(1) errors."""
import numpy as np
import pytest

import pta_inputs as pi

ORDERS = [(0, 1), (1, 1), (2, 7), (2, 16)]


def check(orc, d, c, q, order, nchunk):
    _, _, per = orc.loglike(d, c[None, :], per_psr=True)
    tr = orc.trace(d, c, q)
    r = orc.scan_filter(d, c, q, order, nchunk)
    N = tr["e"].size
    if N == 0:
        assert r["ll"] == 0.0 and r["xs"].size == 0
        return
    sd = np.sqrt(np.einsum("kii->ki", tr["Pf"]))
    assert np.max(np.abs(r["xs"] - tr["x"]) / sd) < 1e-6
    assert np.max(np.abs(r["Ps"] - tr["Pf"]) / (sd[:, :, None] * sd[:, None, :])) < 1e-6
    assert abs(r["ll"] - per[0, q]) <= 3e-9 * abs(per[0, q])


@pytest.mark.parametrize("order,nchunk", ORDERS)
def test_scan_spin_model(oracle_mod, order, nchunk):
    d = pi.make_spin("t", n_toa=120, seed=5)
    for c in d.to_canon(pi.sample_theta(d, 3, 7)):
        check(oracle_mod, d, c, 0, order, nchunk)


@pytest.mark.parametrize("order,nchunk", ORDERS)
def test_scan_per_pulsar_model(oracle_mod, order, nchunk):
    d = pi.make_pta("t", n_psr=4, counts=[150, 1, 0, 90], seed=31)
    for c in d.to_canon(pi.sample_theta(d, 3, 7)):
        for q in range(d.n_psr):
            check(oracle_mod, d, c, q, order, nchunk)


def test_scan_prior_corners(oracle_mod):
    d = pi.make_pta("t", n_psr=1, counts=[400], seed=33)
    for c in d.to_canon(np.array([d.lo, d.hi])):
        for order, nchunk in ORDERS:
            check(oracle_mod, d, c, 0, order, nchunk)
