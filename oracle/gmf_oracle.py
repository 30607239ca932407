"""FP64 CPU oracle for block-wise adaptive SGD of generalized matrix factorization.

TEST INFRASTRUCTURE.  This module is the slow, plain reference that the HIP
library is checked against.  Only the tests, the smoke entry point and the
benchmark's CPU-baseline leg may import it; the product path never does.  It
shares no code with the HIP library: it re-derives every formula from the
paper and re-implements the seeded schedule generator from its published
definition (SplitMix64, Steele, Lea and Flood 2014).

Model (Section 2, eq. 1-3): y_ij follows an exponential dispersion family with
mean mu_ij, g(mu_ij) = eta_ij = x_i' beta_j + gamma_i' z_j + u_i' v_j, and the
penalised negative log-likelihood of eq. 6 is minimised.

Estimator (Section 3.2.2, eq. 11-15, Algorithm 1, Appendix B "stochastic
gradient with non-zero covariate effects"): each step picks a block
B = I x J, forms eta, mu and the first/second derivatives of the deviance on
it, builds unbiased minibatch gradients for [Gamma, U]_I and [B, V]_J, smooths
them with exponential moving averages and takes a bias-corrected diagonal
quasi-Newton step.

Readings of points the paper leaves open (each is a parameter here):
  * D1 = dl/deta = -w (y - mu) / (phi nu(mu) g'(mu)), the derivative of the
    negative log-likelihood (the printed sign is that of the log-likelihood).
  * The ridge terms enter with a + sign (eq. 15), lambda ordered (B, Gamma, U, V).
  * The Hessian of Gamma uses Z*Z (the minibatch form of Appendix B).
  * Bias factor (eq. 11-12): bias_mode 0 uses (1-(1-a2)^t)/(1-(1-a1)^t), the
    Adam form for EMAs with weight a on the new value; bias_mode 1 uses the
    printed (1-a2^t)/(1-a1^t).  t is the global step counter starting at 1.
  * EMA moments start at zero; damping delta is added to the smoothed Hessian.
  * For the log link eta is clamped to [log(eps), eta_max] before the inverse
    link; the identity link is not clamped.
  * Both halves of a step use the pre-step parameters (Algorithm 1 uses V^t in
    its step 4).
  * Partitions are drawn once; each sweep visits J_1..J_S in order and draws
    the row block uniformly with replacement; an epoch is R sweeps (R*S steps).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

# ---------------------------------------------------------------------------
# Families (Section 2, eq. 1-2; Supplementary Table 1; Appendix B for NB)
# ---------------------------------------------------------------------------

FAMILIES = ("poisson", "negbin", "gaussian", "gamma", "bernoulli", "invgauss")


def _xlogy_ratio(y, a):
    """y * log(y / a) with the limit 0 at y = 0."""
    y = np.asarray(y, dtype=np.float64)
    out = np.zeros(np.broadcast(y, a).shape)
    pos = y > 0
    ya = np.broadcast_to(y, out.shape)
    aa = np.broadcast_to(a, out.shape)
    out[pos] = ya[pos] * np.log(ya[pos] / aa[pos])
    return out


def unit_deviance(family: str, y, mu, nb_alpha=5.0):
    """D(y, mu) = -2 log{f(y, mu)/f(y, y)} without the dispersion (Supp. Table 1 x 2).
    nb_alpha may be a scalar or a per-column vector (broadcast over rows)."""
    y = np.asarray(y, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    if family == "gaussian":
        return (y - mu) ** 2
    if family == "poisson":
        return 2.0 * (_xlogy_ratio(y, mu) - (y - mu))
    if family == "negbin":
        a = np.asarray(nb_alpha, dtype=np.float64)
        return 2.0 * (_xlogy_ratio(y, mu) - (y + a) * np.log((y + a) / (mu + a)))
    if family == "gamma":
        return 2.0 * ((y - mu) / mu - np.log(y / mu))
    if family == "invgauss":
        return (y - mu) ** 2 / (y * mu ** 2)
    if family == "bernoulli":
        return 2.0 * (_xlogy_ratio(y, mu) + _xlogy_ratio(1.0 - y, 1.0 - mu))
    raise ValueError(family)


def variance_fn(family: str, mu, nb_alpha=5.0):
    """nu(mu) (Supp. Table 1)."""
    mu = np.asarray(mu, dtype=np.float64)
    if family == "gaussian":
        return np.ones_like(mu)
    if family == "poisson":
        return mu
    if family == "negbin":
        return mu * (1.0 + mu / np.asarray(nb_alpha, dtype=np.float64))
    if family == "gamma":
        return mu ** 2
    if family == "invgauss":
        return mu ** 3
    if family == "bernoulli":
        return mu * (1.0 - mu)
    raise ValueError(family)


def link_deriv(link: str, mu):
    """g'(mu) for g = log, identity or logit."""
    if link == "log":
        return 1.0 / mu
    if link == "identity":
        return np.ones_like(mu)
    if link == "logit":
        return 1.0 / (mu * (1.0 - mu))
    raise ValueError(link)


def inverse_link(link: str, eta, eps: float = 1e-8, eta_max: float = 30.0):
    """mu = g^{-1}(eta) with the clamps: log link eta in [log eps, eta_max],
    logit link eta in [-eta_max, eta_max]."""
    if link == "log":
        return np.exp(np.clip(eta, np.log(eps), eta_max))
    if link == "identity":
        return np.asarray(eta, dtype=np.float64)
    if link == "logit":
        return 1.0 / (1.0 + np.exp(-np.clip(eta, -eta_max, eta_max)))
    raise ValueError(link)


def deviance_derivatives(family, link, y, mu, w, phi, nb_alpha=5.0):
    """First derivative and Fisher weight of the per-entry NLL in eta (Section 3).

    D1 = -w (y - mu) / (phi nu g'),  D2 = w / (phi nu g'^2).
    A missing entry (NaN) is imputed by its mean, y <- mu (Section 3.2.2).
    """
    y = np.where(np.isnan(y), mu, y)
    nu = variance_fn(family, mu, nb_alpha)
    gp = link_deriv(link, mu)
    wt = 1.0 if w is None else w
    D1 = -wt * (y - mu) / (phi * nu * gp)
    D2 = wt / (phi * nu * gp * gp) * np.ones_like(mu)
    return D1, D2


def observed_deviance(family, y, mu, nb_alpha=5.0, w=None):
    """Unit deviances with missing entries (NaN) contributing 0 (y <- mu)."""
    miss = np.isnan(y)
    dev = unit_deviance(family, np.where(miss, mu, y), mu, nb_alpha)
    dev = np.where(miss, 0.0, dev)
    return dev if w is None else w * dev


# ---------------------------------------------------------------------------
# Seeded schedule: SplitMix64 counter streams, Fisher-Yates, block draws
# ---------------------------------------------------------------------------

_M64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15


def _mix64(z: int) -> int:
    z &= _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def stream_key(seed: int, stream: int) -> int:
    """Key of sub-stream ``stream``: the (stream+1)-th SplitMix64 output of ``seed``."""
    return _mix64((seed + (stream + 1) * _GOLDEN) & _M64)


def splitmix_draw(key: int, k: int) -> int:
    """k-th output (k = 0, 1, ...) of the SplitMix64 sequence started at state ``key``."""
    return _mix64((key + (k + 1) * _GOLDEN) & _M64)


def uniform_below(u: int, n: int) -> int:
    """floor(u * n / 2^64): an index in [0, n) from a 64-bit draw."""
    return (u * n) >> 64


def permutation(seed: int, stream: int, n: int) -> np.ndarray:
    """Fisher-Yates shuffle of 0..n-1; step i = n-1..1 uses draw number n-1-i."""
    key = stream_key(seed, stream)
    perm = list(range(n))
    for i in range(n - 1, 0, -1):
        j = uniform_below(splitmix_draw(key, n - 1 - i), i + 1)
        perm[i], perm[j] = perm[j], perm[i]
    return np.asarray(perm, dtype=np.int64)


def partition(perm: np.ndarray, nblocks: int):
    """Split a permutation into nblocks contiguous pieces, piece r = [floor(rN/K), floor((r+1)N/K))."""
    N = len(perm)
    return [perm[(r * N) // nblocks:((r + 1) * N) // nblocks] for r in range(nblocks)]


STREAM_ROWS, STREAM_COLS, STREAM_DRAWS = 0, 1, 2


def row_block_draw(seed: int, t: int, R: int) -> int:
    """Row block of global step t (t = 1, 2, ...): uniform on 0..R-1, with replacement."""
    return uniform_below(splitmix_draw(stream_key(seed, STREAM_DRAWS), t - 1), R)


def col_block_of_step(t: int, S: int) -> int:
    """Column block of global step t: the sweep visits J_1..J_S in order (Algorithm 1)."""
    return (t - 1) % S


# ---------------------------------------------------------------------------
# Configuration and state
# ---------------------------------------------------------------------------


@dataclass
class Config:
    family: str = "poisson"
    link: str = "log"
    phi: float = 1.0
    nb_alpha: float = 5.0
    lam: Sequence[float] = (0.0, 0.0, 1.0, 1.0)   # B, Gamma, U, V
    rate0: float = 0.05
    decay: float = 0.05
    tau: float = 0.75
    alpha1: float = 0.1
    alpha2: float = 0.01
    damping: float = 1e-3
    eps: float = 1e-8
    eta_max: float = 30.0
    bias_mode: int = 0
    R: int = 10
    S: int = 5
    seed: int = 0
    estimate_phi: bool = False     # Appendix B, "Unknown dispersion parameter"
    estimate_alpha: bool = False   # Appendix B, "Negative Binomial inflation parameter"


def learning_rate(cfg: Config, t: int) -> float:
    """rho_t = k0 / (1 + k0 k1 t)^tau (Section 3.2)."""
    return cfg.rate0 / (1.0 + cfg.rate0 * cfg.decay * t) ** cfg.tau


def bias_factor(cfg: Config, t: int) -> float:
    """alpha_t of eq. 11 (see the reading in the module docstring)."""
    a1, a2 = cfg.alpha1, cfg.alpha2
    if cfg.bias_mode == 0:
        return (1.0 - (1.0 - a2) ** t) / (1.0 - (1.0 - a1) ** t)
    return (1.0 - a2 ** t) / (1.0 - a1 ** t)


class OracleGMF:
    """Plain FP64 replay of Algorithm 1 with covariates (Appendix B)."""

    def __init__(self, cfg: Config, Y, X, Z, B0, A0, U0, V0, W=None):
        self.cfg = cfg
        self.Y = np.asarray(Y, dtype=np.float64)
        self.n, self.m = self.Y.shape
        self.X = np.asarray(X, dtype=np.float64).reshape(self.n, -1)
        self.Z = np.asarray(Z, dtype=np.float64).reshape(self.m, -1)
        self.p, self.q = self.X.shape[1], self.Z.shape[1]
        self.B = np.array(B0, dtype=np.float64).reshape(self.m, self.p)
        self.A = np.array(A0, dtype=np.float64).reshape(self.n, self.q)
        self.U = np.array(U0, dtype=np.float64)
        self.V = np.array(V0, dtype=np.float64)
        self.d = self.U.shape[1]
        self.W = None if W is None else np.asarray(W, dtype=np.float64)
        # smoothed gradients/Hessians for [Gamma, U] (rows) and [B, V] (columns)
        self.Grow = np.zeros((self.n, self.q + self.d))
        self.Hrow = np.zeros((self.n, self.q + self.d))
        self.Gcol = np.zeros((self.m, self.p + self.d))
        self.Hcol = np.zeros((self.m, self.p + self.d))
        self.t = 0
        self.row_perm = permutation(cfg.seed, STREAM_ROWS, self.n)
        self.col_perm = permutation(cfg.seed, STREAM_COLS, self.m)
        self.row_blocks = partition(self.row_perm, cfg.R)
        self.col_blocks = partition(self.col_perm, cfg.S)
        lam = cfg.lam
        self.lam_row = np.array([lam[1]] * self.q + [lam[2]] * self.d)
        self.lam_col = np.array([lam[0]] * self.p + [lam[3]] * self.d)
        self.last_block_dev = None
        # dispersion and NB shape in use: fixed, or the smoothed stochastic
        # estimates of Appendix B started at the configured values
        self.phi_bar = float(cfg.phi)
        self.alpha_bar = cfg.nb_alpha if np.ndim(cfg.nb_alpha) == 0 else np.asarray(
            cfg.nb_alpha, dtype=np.float64)

    def alpha_of(self, J=None):
        """NB shape of the columns J (scalar, or the per-column values)."""
        a = self.alpha_bar
        return a if np.ndim(a) == 0 or J is None else a[J]

    def estimate_dispersion(self, t, yB, mu, wB, aJ, ns, ms):
        """Stochastic dispersion and NB-shape updates of Appendix B from the
        block's pre-step means, over the observed entries: Pearson estimate
        phi^ = (1/N) (nm/(n* m*)) sum w (y - mu)^2 / nu(mu) with
        N = nm - mp - nq - (n+m)d - 1, moment estimate alpha^ = sum w mu^2 /
        sum w ((y - mu)^2 - mu); each smoothed with weight rho_t,
        alpha_bar <- (1 - rho_t) alpha_bar + rho_t max(eps, alpha^)."""
        cfg = self.cfg
        obs = ~np.isnan(yB)
        wt = np.ones_like(mu) if wB is None else wB
        y0 = np.where(obs, yB, mu)
        rho = learning_rate(cfg, t)
        if cfg.estimate_phi:
            N = (self.n * self.m - self.m * self.p - self.n * self.q
                 - (self.n + self.m) * self.d - 1)
            pear = np.where(obs, wt * (y0 - mu) ** 2 / variance_fn(cfg.family, mu, aJ), 0.0)
            phi_hat = (self.n * self.m) / (ns * ms) * pear.sum() / N
            self.phi_bar = (1.0 - rho) * self.phi_bar + rho * phi_hat
        if cfg.estimate_alpha:
            num = np.where(obs, wt * mu * mu, 0.0).sum()
            den = np.where(obs, wt * ((y0 - mu) ** 2 - mu), 0.0).sum()
            alpha_hat = num / den
            self.alpha_bar = (1.0 - rho) * self.alpha_bar + rho * max(cfg.eps, alpha_hat)

    # -- one step ----------------------------------------------------------
    def block_of_step(self, t: int):
        r = row_block_draw(self.cfg.seed, t, self.cfg.R)
        s = col_block_of_step(t, self.cfg.S)
        return r, s

    def step(self) -> float:
        """Advance t by one and apply Algorithm 1 steps 1-4 to block (r_t, s_t)."""
        t = self.t + 1
        r, s = self.block_of_step(t)
        return self.step_block(t, r, s)

    def step_block(self, t: int, r: int, s: int) -> float:
        """Steps 2-4 of Algorithm 1 on block I_r x J_s with counter t."""
        cfg = self.cfg
        I = self.row_blocks[r]
        J = self.col_blocks[s]
        ns, ms = len(I), len(J)
        # step 2: eta, mu, derivatives on the block (eq. 3, Section 3)
        eta = (self.X[I] @ self.B[J].T + self.A[I] @ self.Z[J].T
               + self.U[I] @ self.V[J].T)
        mu = inverse_link(cfg.link, eta, cfg.eps, cfg.eta_max)
        yB = self.Y[np.ix_(I, J)]
        wB = None if self.W is None else self.W[np.ix_(I, J)]
        aJ = self.alpha_of(J)
        D1, D2 = deviance_derivatives(cfg.family, cfg.link, yB, mu, wB, self.phi_bar, aJ)
        # minibatch gradients from the pre-step parameters (eq. 15, Appendix B)
        Pc = np.hstack([self.Z[J], self.V[J]])            # [Z, V]_J
        Pr = np.hstack([self.X[I], self.U[I]])            # [X, U]_I
        row_par = np.hstack([self.A[I], self.U[I]])       # [Gamma, U]_I
        col_par = np.hstack([self.B[J], self.V[J]])       # [B, V]_J
        G_row = (self.m / ms) * (D1 @ Pc) + self.lam_row * row_par
        H_row = (self.m / ms) * (D2 @ (Pc * Pc)) + self.lam_row
        G_col = (self.n / ns) * (D1.T @ Pr) + self.lam_col * col_par
        H_col = (self.n / ns) * (D2.T @ (Pr * Pr)) + self.lam_col
        # exponential moving averages on the touched rows (eq. 12)
        a1, a2 = cfg.alpha1, cfg.alpha2
        self.Grow[I] = (1 - a1) * self.Grow[I] + a1 * G_row
        self.Hrow[I] = (1 - a2) * self.Hrow[I] + a2 * H_row
        self.Gcol[J] = (1 - a1) * self.Gcol[J] + a1 * G_col
        self.Hcol[J] = (1 - a2) * self.Hcol[J] + a2 * H_col
        # bias-corrected diagonal quasi-Newton step (eq. 13-14)
        scale = learning_rate(cfg, t) * bias_factor(cfg, t)
        row_new = row_par - scale * self.Grow[I] / (self.Hrow[I] + cfg.damping)
        col_new = col_par - scale * self.Gcol[J] / (self.Hcol[J] + cfg.damping)
        q, p = self.q, self.p
        self.A[I] = row_new[:, :q]
        self.U[I] = row_new[:, q:]
        self.B[J] = col_new[:, :p]
        self.V[J] = col_new[:, p:]
        self.t = t
        self.last_block_dev = float(np.sum(observed_deviance(cfg.family, yB, mu, aJ, wB)))
        if cfg.estimate_phi or cfg.estimate_alpha:
            self.estimate_dispersion(t, yB, mu, wB, aJ, ns, ms)
        return self.last_block_dev

    def steps(self, k: int):
        return [self.step() for _ in range(k)]

    def epoch(self):
        return self.steps(self.cfg.R * self.cfg.S)

    # -- monitors ------------------------------------------------------------
    def eta_full(self, rows=None):
        rows = np.arange(self.n) if rows is None else rows
        return (self.X[rows] @ self.B.T + self.A[rows] @ self.Z.T
                + self.U[rows] @ self.V.T)

    def full_deviance(self, chunk=4096) -> float:
        """sum_ij w_ij D(y_ij, mu_ij) over the whole matrix."""
        cfg = self.cfg
        tot = 0.0
        for r0 in range(0, self.n, chunk):
            rows = np.arange(r0, min(self.n, r0 + chunk))
            mu = inverse_link(cfg.link, self.eta_full(rows), cfg.eps, cfg.eta_max)
            dev = observed_deviance(cfg.family, self.Y[rows], mu, self.alpha_of(None),
                                    None if self.W is None else self.W[rows])
            tot += float(dev.sum())
        return tot

    def objective(self) -> float:
        """Penalised NLL up to a constant: D/(2 phi) + sum lambda/2 ||.||_F^2 (eq. 6)."""
        lam = self.cfg.lam
        pen = 0.5 * (lam[0] * np.sum(self.B ** 2) + lam[1] * np.sum(self.A ** 2)
                     + lam[2] * np.sum(self.U ** 2) + lam[3] * np.sum(self.V ** 2))
        return self.full_deviance() / (2.0 * self.phi_bar) + pen

    def full_gradient(self):
        """Exact gradient of the objective: D1 [Z,V] + lam[0,U], D1' [X,U] + lam[0,V]."""
        cfg = self.cfg
        mu = inverse_link(cfg.link, self.eta_full(), cfg.eps, cfg.eta_max)
        D1, _ = deviance_derivatives(cfg.family, cfg.link, self.Y, mu, self.W,
                                     self.phi_bar, self.alpha_of(None))
        g_row = D1 @ np.hstack([self.Z, self.V]) + self.lam_row * np.hstack([self.A, self.U])
        g_col = D1.T @ np.hstack([self.X, self.U]) + self.lam_col * np.hstack([self.B, self.V])
        return g_row, g_col

    def params(self):
        return self.B.copy(), self.A.copy(), self.U.copy(), self.V.copy()


# ---------------------------------------------------------------------------
# Identifiability post-processing (Algorithm 2, constraints (A) and (B1))
# ---------------------------------------------------------------------------


def postprocess_A_B1(X, Z, B, A, U, V):
    """Project (B, Gamma, U, V) onto constraints (A) then (B1) (Algorithm 2).

    (A): Gamma, U projected off span(X) (B absorbs the change), then V off
    span(Z) (Gamma absorbs it).  (B1): U V' = P S Q' by SVD; U <- P S, V <- Q,
    and each column of V has its first non-zero entry positive.
    """
    X = np.asarray(X, np.float64)
    Z = np.asarray(Z, np.float64)
    B, A, U, V = (np.array(a, np.float64) for a in (B, A, U, V))
    p, q, d = X.shape[1], Z.shape[1], U.shape[1]
    if p > 0:
        DG = np.linalg.solve(X.T @ X, X.T @ A)
        A = A - X @ DG
        B = B + Z @ DG.T
        DU = np.linalg.solve(X.T @ X, X.T @ U)
        U = U - X @ DU
        B = B + V @ DU.T
    if q > 0:
        DV = np.linalg.solve(Z.T @ Z, Z.T @ V)
        V = V - Z @ DV
        A = A + U @ DV.T
    P, s, Qt = np.linalg.svd(U @ V.T, full_matrices=False)
    U = P[:, :d] * s[:d]
    V = Qt[:d].T.copy()
    for k in range(d):
        nz = np.nonzero(V[:, k])[0]
        if len(nz) and V[nz[0], k] < 0:
            V[:, k] = -V[:, k]
            U[:, k] = -U[:, k]
    return B, A, U, V


# ---------------------------------------------------------------------------
# Projection of new rows with the column side frozen (row half of Algorithm 1)
# ---------------------------------------------------------------------------


def project_rows(cfg: Config, Ynew, Xnew, Z, B, V, A0, U0, epochs: int,
                 col_blocks, W=None, record=None):
    """Row-side aSGD for new rows: B, V frozen; each step uses all new rows and
    column block J_{(t-1) mod S}; t restarts at 1; moments start at zero."""
    Y = np.asarray(Ynew, np.float64)
    n, m = Y.shape
    X = np.asarray(Xnew, np.float64).reshape(n, -1)
    Z = np.asarray(Z, np.float64).reshape(m, -1)
    B = np.asarray(B, np.float64).reshape(m, -1)
    V = np.asarray(V, np.float64)
    A = np.array(A0, np.float64).reshape(n, -1)
    U = np.array(U0, np.float64)
    q, d = A.shape[1], U.shape[1]
    lam_row = np.array([cfg.lam[1]] * q + [cfg.lam[2]] * d)
    G = np.zeros((n, q + d))
    H = np.zeros((n, q + d))
    S = len(col_blocks)
    t = 0
    for _ in range(epochs * S):
        t += 1
        J = col_blocks[(t - 1) % S]
        ms = len(J)
        eta = X @ B[J].T + A @ Z[J].T + U @ V[J].T
        mu = inverse_link(cfg.link, eta, cfg.eps, cfg.eta_max)
        wB = None if W is None else W[:, J]
        D1, D2 = deviance_derivatives(cfg.family, cfg.link, Y[:, J], mu, wB,
                                      cfg.phi, cfg.nb_alpha)
        Pc = np.hstack([Z[J], V[J]])
        par = np.hstack([A, U])
        Gh = (m / ms) * (D1 @ Pc) + lam_row * par
        Hh = (m / ms) * (D2 @ (Pc * Pc)) + lam_row
        G = (1 - cfg.alpha1) * G + cfg.alpha1 * Gh
        H = (1 - cfg.alpha2) * H + cfg.alpha2 * Hh
        par = par - learning_rate(cfg, t) * bias_factor(cfg, t) * G / (H + cfg.damping)
        A, U = par[:, :q], par[:, q:]
        if record is not None:
            record.append((A.copy(), U.copy()))
    return A, U


def row_deviance(cfg: Config, Y, X, Z, B, A, U, V, W=None):
    """Per-row deviance sum_j w_ij D(y_ij, mu_ij)."""
    eta = (np.asarray(X) @ np.asarray(B).T + np.asarray(A) @ np.asarray(Z).T
           + np.asarray(U) @ np.asarray(V).T)
    mu = inverse_link(cfg.link, eta, cfg.eps, cfg.eta_max)
    return observed_deviance(cfg.family, np.asarray(Y, np.float64), mu, cfg.nb_alpha,
                             W).sum(axis=1)


# ---------------------------------------------------------------------------
# Out-of-sample reconstruction error (Section 5.2)
# ---------------------------------------------------------------------------


def heldout_metrics(family, y_val, mu_val, ybar_train, nb_alpha=5.0):
    """The two relative out-of-sample errors of Section 5.2 over the held-out
    entries: the relative squared logarithmic error
    sum [log((1+y)/(1+mu))]^2 / sum [log((1+y)/(1+ybar_T))]^2, and the relative
    deviance sum D(y, mu) / sum D(y, ybar_T), ybar_T the mean of the training
    entries; the deviance is the Poisson one (the paper's) and, as a second
    value, the model family's.  Returns (log_error, poisson_deviance,
    family_deviance)."""
    y = np.asarray(y_val, np.float64)
    mu = np.asarray(mu_val, np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):   # count metrics of real data: NaN
        log_err = (np.sum(np.log((1.0 + y) / (1.0 + mu)) ** 2)
                   / np.sum(np.log((1.0 + y) / (1.0 + ybar_train)) ** 2))
        pois = (np.sum(unit_deviance("poisson", y, mu))
                / np.sum(unit_deviance("poisson", y, np.full_like(y, ybar_train))))
    fam = (np.sum(unit_deviance(family, y, mu, nb_alpha))
           / np.sum(unit_deviance(family, y, np.full_like(y, ybar_train), nb_alpha)))
    return log_err, pois, fam


# ---------------------------------------------------------------------------
# Starting values of projected rows (learned warm start with per-row fallback)
# ---------------------------------------------------------------------------


def row_intercept_start(cfg: Config, Y, X, B, q: int):
    """Gamma_0 of new rows given the frozen X B' part, with the first column of
    Z the intercept: the row intercept that matches the row total when U = 0,
    log link sum_j exp(x_i' beta_j + g) = sum_j y_ij + 1/2, identity link
    sum_j (x_i' beta_j + g) = sum_j y_ij.  Other columns of Gamma are 0."""
    Y = np.asarray(Y, np.float64)
    n, m = Y.shape
    eta_x = np.asarray(X, np.float64).reshape(n, -1) @ np.asarray(B, np.float64).reshape(m, -1).T
    A0 = np.zeros((n, q))
    if q == 0:
        return A0
    if cfg.link == "log":
        mu_x = inverse_link("log", eta_x, cfg.eps, cfg.eta_max)
        A0[:, 0] = np.log(Y.sum(axis=1) + 0.5) - np.log(mu_x.sum(axis=1))
    else:
        A0[:, 0] = (Y.sum(axis=1) - eta_x.sum(axis=1)) / m
    return A0


def warm_start_rows(cfg: Config, Y, X, Z, B, V, A0, U_cand):
    """Per row, start from U_cand's row if its row deviance (with A0) is below
    that of u_i = 0, else from 0.  Returns (U0, warm mask, dev_cand, dev_zero)."""
    U_cand = np.asarray(U_cand, np.float64)
    dev_c = row_deviance(cfg, Y, X, Z, B, A0, U_cand, V)
    dev_0 = row_deviance(cfg, Y, X, Z, B, A0, np.zeros_like(U_cand), V)
    warm = dev_c < dev_0
    U0 = np.where(warm[:, None], U_cand, 0.0)
    return U0, warm, dev_c, dev_0
