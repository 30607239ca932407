"""FP64 oracle of the paper's parameter initialization (Section 4.1,
"Parameter initialization"), in its least-squares form for high-dimensional
data.

TEST INFRASTRUCTURE.  Only the tests, the smoke entry point and the
benchmark's CPU-baseline leg may import it; the product path never does.  It
shares no code with the HIP library.

Steps, in the paper's order:
  1. Column effects: the m regressions of the link-transformed response
     L = g(y + c) on X, by ordinary least squares (the approximation the paper
     gives for the m column GLMs): B' = argmin ||L - X B'||_F.
  2. Row effects: given the offsets X B', the n regressions of the residual on
     Z, by least squares: Gamma = argmin ||(L - X B') - Gamma Z'||_F.
  3. Latent scores: the first d left singular vectors of the residual matrix
     at mu~ = g^-1(X B' + Gamma Z'), Pearson residuals (y - mu~)/sqrt(nu(mu~))
     (or deviance residuals sign(y - mu~) sqrt(D(y, mu~))), by a randomized
     range finder with power iterations (Halko, Martinsson and Tropp 2011,
     Algorithms 4.4 and 5.1) from a caller-supplied Gaussian test matrix Omega
     (m x k, k >= d): Y0 = E Omega; q times: Q = orth(Y), Y = E orth(E' Q);
     Q = orth(Y); the left singular vectors of Q' E, mapped back by Q.
  4. Loadings: the m column regressions of the link-scale residual
     R = L - X B' - Gamma Z' on the scores (the least-squares form of the
     column GLMs with the scores as design and the offsets in the predictor):
     V' = argmin ||R - U V'||_F.

Readings (the paper is silent on these points):
  * c = 1/2 for the log link (g(0) is not finite), 0 for the identity link;
    the logit link transforms (y + c)/(1 + 2c) with c = 1/2.
  * Missing entries (NaN) take the current prediction: in step 1 the mean of
    the column's observed L, afterwards a zero residual (y <- mu).
  * The scores are scaled so that each pair of columns (u_k, v_k) has equal
    Euclidean norms, which leaves U V' unchanged and minimises
    ||u_k||^2 + ||v_k||^2 over the rescalings of the pair (the ridge penalty
    of eq. 6 with lambda_U = lambda_V).
  * Weights multiply the residuals of step 3 (sqrt(w) for Pearson, w inside
    the deviance); the least-squares steps are unweighted.
  * mu~ is clamped like the fit's mean (eta in [log eps, eta_max], log link).
"""
from __future__ import annotations

import numpy as np

from oracle import gmf_oracle as G


def link_offset(link: str, offset=None) -> float:
    if offset is not None and offset >= 0:
        return float(offset)
    return 0.0 if link == "identity" else 0.5


def link_transform(link: str, Y, offset=None):
    """L = g(y + c); for the logit link g((y + c)/(1 + 2c)), which maps {0, 1}
    into (0, 1)."""
    c = link_offset(link, offset)
    Y = np.asarray(Y, np.float64)
    if link == "log":
        return np.log(Y + c)
    if link == "identity":
        return Y + c
    if link == "logit":
        q = (Y + c) / (1.0 + 2.0 * c)
        return np.log(q / (1.0 - q))
    raise ValueError(link)


def residuals(kind: str, family: str, Y, mu, nb_alpha: float = 5.0, W=None):
    """Pearson (y - mu)/sqrt(nu(mu)/w) or deviance sign(y - mu) sqrt(w D(y, mu))."""
    Y = np.asarray(Y, np.float64)
    w = 1.0 if W is None else np.asarray(W, np.float64)
    if kind == "pearson":
        return (Y - mu) * np.sqrt(w / G.variance_fn(family, mu, nb_alpha))
    if kind == "deviance":
        D = np.maximum(G.unit_deviance(family, Y, mu, nb_alpha), 0.0)
        return np.sign(Y - mu) * np.sqrt(w * D)
    raise ValueError(kind)


def _orth(M):
    Q, _ = np.linalg.qr(M)
    return Q


def _range_basis(E, Omega, power_iters: int):
    Yk = E @ Omega
    for _ in range(power_iters):
        Q = _orth(Yk)
        Yk = E @ _orth(E.T @ Q)
    return _orth(Yk)


def randomized_left_vectors(E, Omega, power_iters: int, d: int):
    """First d left singular vectors of E (n x m) from the test matrix Omega."""
    Q = _range_basis(E, Omega, power_iters)
    Ub, _, _ = np.linalg.svd(Q.T @ E, full_matrices=False)
    return Q @ Ub[:, :d]


def randomized_singular_values(E, Omega, power_iters: int):
    """The singular values of Q'E, the range finder's estimates of the k
    leading singular values of E (exact for the leading ones when the power
    iterations have converged; below the true values in a flat tail)."""
    Q = _range_basis(E, Omega, power_iters)
    return np.linalg.svd(Q.T @ E, compute_uv=False)


def initialize(cfg: G.Config, Y, X, Z, d: int, Omega, power_iters: int = 2,
               residual: str = "pearson", offset=None, W=None):
    """(B, Gamma, U, V) of the least-squares initialization."""
    Y = np.asarray(Y, np.float64)
    n, m = Y.shape
    X = np.asarray(X, np.float64).reshape(n, -1)
    Z = np.asarray(Z, np.float64).reshape(m, -1)
    p, q = X.shape[1], Z.shape[1]
    L = link_transform(cfg.link, Y, offset)
    # a missing entry takes the current prediction: before any effect is
    # fitted, the mean of its column's observed L; afterwards its residuals
    # are 0 (y <- mu)
    miss = np.isnan(Y)
    L1 = np.where(miss, np.nanmean(L, axis=0), L) if miss.any() else L
    # 1. column effects
    if p > 0:
        B = np.linalg.lstsq(X, L1, rcond=None)[0].T
    else:
        B = np.zeros((m, 0))
    R1 = np.where(miss, 0.0, L1 - X @ B.T)
    # 2. row effects given the column offsets
    if q > 0:
        A = np.linalg.lstsq(Z, R1.T, rcond=None)[0].T
    else:
        A = np.zeros((n, 0))
    eta0 = X @ B.T + A @ Z.T
    mu0 = G.inverse_link(cfg.link, eta0, cfg.eps, cfg.eta_max)
    # 3. scores: leading left singular vectors of the residual matrix
    E = np.where(miss, 0.0, residuals(residual, cfg.family, np.where(miss, mu0, Y), mu0,
                                      cfg.nb_alpha, W))
    U = randomized_left_vectors(E, np.asarray(Omega, np.float64), power_iters, d)
    # 4. loadings: least squares of the link-scale residual on the scores
    R = np.where(miss, 0.0, L - eta0)
    V = np.linalg.lstsq(U, R, rcond=None)[0].T
    # equal norms within each pair (u_k, v_k)
    nu = np.linalg.norm(U, axis=0)
    nv = np.linalg.norm(V, axis=0)
    s = np.sqrt(np.where(nu > 0, nv / np.where(nu > 0, nu, 1.0), 1.0))
    s = np.where(s > 0, s, 1.0)
    return B, A, U * s, V / s
