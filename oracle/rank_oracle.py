"""FP64 oracle of the rank selection of Section 4.2 ("Model selection").

TEST INFRASTRUCTURE.  Only the tests, the smoke entry point and the
benchmark's CPU-baseline leg may import it; the product path never does.  It
shares no code with the HIP library.

Two criteria, as the paper uses them:
  * spectral thresholding: the eigenvalues (squared singular values) of the
    residual matrix of the initialization (deviance or Pearson residuals after
    the least-squares column and row effects), read by the eigenvalue-gap
    ("edge distribution") estimator of Onatski (2010, Review of Economics and
    Statistics 92(4)): with r_max the largest rank considered, start at
    j = r_max + 1; regress lambda_j .. lambda_{j+4} on a constant and
    (j-1)^{2/3} .. (j+3)^{2/3}, delta = 2 |slope|; r = the largest i <= r_max
    with lambda_i - lambda_{i+1} >= delta (0 if none); j = r + 1; repeat until
    r no longer changes.
  * out-of-sample error: fit every candidate rank with a fold of entries held
    out as missing values and evaluate the held-out deviance (Section 5.2's
    relative deviance); the selected rank minimises the mean over folds.
"""
from __future__ import annotations

import numpy as np

from oracle import gmf_oracle as G


def eigengap_rank(eigenvalues, rmax: int, max_iter: int = 100) -> int:
    """Onatski's edge-distribution estimator on eigenvalues sorted descending
    (at least rmax + 5 of them)."""
    lam = np.asarray(eigenvalues, np.float64)
    if len(lam) < rmax + 5:
        raise ValueError("need at least rmax + 5 eigenvalues")
    j = rmax + 1
    r_prev = -1
    r = 0
    for _ in range(max_iter):
        idx = np.arange(j, j + 5)                       # 1-based indices j .. j+4
        x = (idx - 1.0) ** (2.0 / 3.0)
        y = lam[idx - 1]
        slope = np.polyfit(x, y, 1)[0]
        delta = 2.0 * abs(slope)
        gaps = lam[:rmax] - lam[1:rmax + 1]             # lambda_i - lambda_{i+1}, i = 1..rmax
        above = np.nonzero(gaps >= delta)[0]
        r = int(above[-1] + 1) if len(above) else 0
        if r == r_prev:
            break
        r_prev = r
        j = r + 1
    return r


def cv_deviance(cfg: G.Config, Y, X, Z, B0, A0, U0, V0, heldout, epochs: int):
    """Fit with the held-out entries missing, then Section 5.2's relative
    deviances on them: (log error, Poisson deviance ratio, family deviance
    ratio)."""
    Y = np.asarray(Y, np.float64)
    Ytr = np.where(heldout, np.nan, Y)
    o = G.OracleGMF(cfg, Ytr, X, Z, B0, A0, U0, V0)
    for _ in range(epochs):
        o.epoch()
    mu = G.inverse_link(cfg.link, o.eta_full(), cfg.eps, cfg.eta_max)
    ybar = np.nanmean(Ytr)
    return G.heldout_metrics(cfg.family, Y[heldout], mu[heldout], ybar, cfg.nb_alpha)
