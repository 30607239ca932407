"""Pins of the rank-selection oracle (Section 4.2): the eigenvalue-gap
estimator recovers the number of planted factors of random matrices and finds
none in pure noise, is invariant to the scale of the eigenvalues, follows its
calibration when the largest gap is not the last one; the out-of-sample
deviance of a fit is smallest near the planted rank."""
import numpy as np
import pytest

from oracle import gmf_oracle as G
from oracle import rank_oracle as K


def _spectrum(n, m, d, strength, seed):
    rng = np.random.default_rng(seed)
    E = rng.normal(size=(n, m))
    if d:
        P = np.linalg.qr(rng.normal(size=(n, d)))[0]
        Q = np.linalg.qr(rng.normal(size=(m, d)))[0]
        E += (P * (strength * np.sqrt(n * m) * np.linspace(1.0, 0.6, d))) @ Q.T
    return np.linalg.svd(E, compute_uv=False) ** 2


@pytest.mark.parametrize("d,seed", [(0, 1), (1, 2), (3, 3), (6, 4)])
def test_eigengap_recovers_planted_factors(d, seed):
    lam = _spectrum(600, 300, d, 0.35, seed)
    assert K.eigengap_rank(lam, rmax=12) == d


def test_eigengap_is_scale_invariant():
    lam = _spectrum(500, 250, 4, 0.3, 5)
    assert K.eigengap_rank(lam, 10) == K.eigengap_rank(1e-6 * lam, 10) == \
        K.eigengap_rank(1e4 * lam, 10) == 4


def test_eigengap_takes_the_last_gap_above_threshold():
    """Two groups of spikes: the largest gap follows the first group, but the
    estimator counts every eigenvalue above the bulk's edge."""
    lam = _spectrum(600, 300, 0, 0.0, 6)
    lam = np.concatenate([[900.0 * lam[0], 800.0 * lam[0], 3.0 * lam[0], 2.8 * lam[0]], lam])
    assert K.eigengap_rank(lam, 10) == 4


def test_heldout_deviance_is_smallest_at_the_planted_rank():
    """A Gaussian matrix of rank 3 plus noise, 20 % of its entries held out:
    the held-out relative deviance falls steeply up to rank 3 and rises
    beyond it (overfitting)."""
    rng = np.random.default_rng(5)
    n, m, d = 200, 150, 3
    X, Z = np.ones((n, 1)), np.ones((m, 1))
    Y = rng.normal(size=(n, d)) @ rng.normal(size=(m, d)).T + 0.5 * rng.normal(size=(n, m)) + 1.0
    held = rng.random(size=Y.shape) < 0.2
    cfg = G.Config(family="gaussian", link="identity", R=2, S=2, seed=9, lam=(0, 0, 0.1, 0.1),
                   rate0=0.3, decay=0.05)
    devs = {}
    for dd in (1, 2, 3, 4, 6, 9):
        r = np.random.default_rng(100 + dd)
        devs[dd] = K.cv_deviance(cfg, Y, X, Z, np.ones((m, 1)), np.zeros((n, 1)),
                                 r.normal(0, 0.1, size=(n, dd)), r.normal(0, 0.1, size=(m, dd)),
                                 held, 40)[2]
    assert min(devs, key=devs.get) == 3
    assert devs[2] > 2 * devs[3] and devs[9] > devs[6] > devs[4] > devs[3]
