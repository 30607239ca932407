"""Seeded generators of single-cell-shaped count matrices and starting values.

Every array is drawn from numpy's PCG64 with a fixed seed.  Real-valued inputs
(covariates, starting values) are rounded to float32 so that a float32 device
copy and a float64 host copy hold the same numbers.

Recipes (they stand in for the paper's splatter simulations and its real data,
which are not available; shapes follow the paper's settings):

* ``gen_poisson_small``: Poisson counts, log link, a column intercept through a
  ones column in X and a row intercept through a ones column in Z, latent
  scores and loadings N(0, 0.5^2).
* ``gen_nb``: negative binomial counts (shape alpha), log link, X = [1, batch
  indicator, N(0,1) covariate], Z = 1, with the intercept shift bisected so that
  the expected fraction of zeros is ``zero_frac``.
* ``gen_gaussian_lowrank``: a dense real matrix with a planted low-rank part and
  a clear spectral gap, for the Gaussian / identity-link case.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@dataclass
class Problem:
    family: str                 # "poisson" | "negbin" | "gaussian"
    link: str                   # "log" | "identity"
    n: int
    m: int
    d: int
    p: int
    q: int
    R: int                      # number of row blocks
    S: int                      # number of column blocks
    Y: np.ndarray               # n x m; int32 counts or float64 reals
    X: np.ndarray               # n x p row covariates (float32-representable)
    Z: np.ndarray               # m x q column covariates
    B0: np.ndarray              # m x p starting coefficients
    A0: np.ndarray              # n x q starting coefficients (Gamma)
    U0: np.ndarray              # n x d starting scores
    V0: np.ndarray              # m x d starting loadings
    phi: float = 1.0
    nb_alpha: float = 5.0
    W: Optional[np.ndarray] = None
    sched_seed: int = 0
    true: dict = field(default_factory=dict)
    name: str = ""

    @property
    def k(self) -> int:
        return self.p + self.q + self.d


def _start_values(rng, Y, X, Z, d, family, scale=0.1):
    """Starting values: B's first column from column means of Y, the rest 0."""
    n, m = Y.shape
    p, q = X.shape[1], Z.shape[1]
    B0 = np.zeros((m, p))
    colmean = Y.mean(axis=0)
    if family == "gaussian":
        B0[:, 0] = colmean
    else:
        B0[:, 0] = np.log(colmean + 0.5)
    A0 = np.zeros((n, q))
    U0 = rng.normal(0.0, scale, size=(n, d))
    V0 = rng.normal(0.0, scale, size=(m, d))
    return _f32(B0), _f32(A0), _f32(U0), _f32(V0)


def gen_poisson_small(n=1000, m=500, d=5, R=10, S=5, seed=1001):
    """Poisson, log link, intercepts only (p = q = 1)."""
    rng = _rng(seed)
    X = np.ones((n, 1))
    Z = np.ones((m, 1))
    beta0 = rng.normal(0.0, 1.0, size=(m, 1))
    gamma0 = rng.normal(0.0, 0.5, size=(n, 1))
    U = rng.normal(0.0, 0.5, size=(n, d))
    V = rng.normal(0.0, 0.5, size=(m, d))
    eta = X @ beta0.T + gamma0 @ Z.T + U @ V.T
    Y = rng.poisson(np.exp(eta)).astype(np.int32)
    B0, A0, U0, V0 = _start_values(_rng(seed + 2000), Y, X, Z, d, "poisson")
    return Problem("poisson", "log", n, m, d, 1, 1, R, S, Y, X, Z, B0, A0, U0,
                   V0, sched_seed=seed + 1000, name=f"poisson_{n}x{m}_d{d}",
                   true=dict(B=beta0, A=gamma0, U=U, V=V))


_PAR_THRESHOLD = 100_000_000   # matrices with more entries are sampled in parallel


def _sample_chunk(par, r0, r1, k):
    """Counts of rows r0..r1 (chunk k): own PCG64 stream seeded with (seed, k)."""
    mu = np.exp(par["X"][r0:r1] @ par["B"].T + par["G"][r0:r1] @ par["Z"].T
                + par["U"][r0:r1] @ par["V"].T)
    rng = np.random.Generator(np.random.PCG64([par["seed"], k]))
    if par["family"] == "negbin":
        a = par["alpha"]
        return rng.negative_binomial(a, a / (a + mu)).astype(np.int32)
    return rng.poisson(mu).astype(np.int32)


def _parallel_counts(Y, par, chunk_rows):
    """Fill Y by row chunks of `chunk_rows` in a thread pool (numpy's samplers
    release the GIL); chunk k always draws from the stream (seed, k), so the
    result does not depend on the number of threads.  Threads rather than
    processes: callers may already hold a GPU context, which must not be
    duplicated into forked children."""
    from concurrent.futures import ThreadPoolExecutor
    n = Y.shape[0]
    jobs = [(r0, min(n, r0 + chunk_rows), k) for k, r0 in enumerate(range(0, n, chunk_rows))]

    def run(job):
        r0, r1, k = job
        Y[r0:r1] = _sample_chunk(par, r0, r1, k)

    workers = max(1, min(16, (os.cpu_count() or 1)))
    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(run, jobs))


def _nb_zero_frac(eta, alpha):
    mu = np.exp(eta)
    return float(np.mean((alpha / (alpha + mu)) ** alpha))


def gen_nb(n=10_000, m=2_000, d=10, R=10, S=5, alpha=5.0, zero_frac=0.85,
           seed=1002, family="negbin", calib_rows=2000, chunk_rows=4096, chunked=None):
    """Negative binomial (or Poisson with the same mean) single-cell-shaped data.

    X = [1, b, x] with b a batch indicator for a seeded half of the rows and
    x ~ N(0, 1); Z = 1.  The intercept shift c is bisected on a seeded subset
    of rows so that the expected zero fraction equals ``zero_frac``.  Counts are
    drawn from one stream in row order, or (``chunked``, the default above 1e8
    entries) in row chunks with a stream per chunk, in parallel.
    """
    rng = _rng(seed)
    batch = np.zeros(n)
    batch[rng.permutation(n)[: n // 2]] = 1.0
    X = _f32(np.column_stack([np.ones(n), batch, rng.normal(0.0, 1.0, size=n)]))
    Z = np.ones((m, 1))
    B_rest = np.column_stack([rng.normal(0.0, 1.0, size=m),
                              rng.normal(0.0, 0.5, size=m),
                              rng.normal(0.0, 0.25, size=m)])
    gamma0 = rng.normal(0.0, 0.5, size=(n, 1))
    U = rng.normal(0.0, 0.5, size=(n, d))
    V = rng.normal(0.0, 0.5, size=(m, d))

    sub = _rng(seed + 7).choice(n, size=min(calib_rows, n), replace=False)

    def eta_rows(rows, c):
        B = B_rest.copy()
        B[:, 0] += c
        return X[rows] @ B.T + gamma0[rows] @ Z.T + U[rows] @ V.T

    lo, hi = -15.0, 10.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if family == "negbin":
            zf = _nb_zero_frac(eta_rows(sub, mid), alpha)
        else:
            zf = float(np.mean(np.exp(-np.exp(eta_rows(sub, mid)))))
        if zf > zero_frac:
            lo = mid
        else:
            hi = mid
    c = 0.5 * (lo + hi)
    B = B_rest.copy()
    B[:, 0] += c

    Y = np.empty((n, m), dtype=np.int32)
    if chunked is None:
        chunked = n * m >= _PAR_THRESHOLD
    if not chunked:
        yr = _rng(seed + 11)
        for r0 in range(0, n, chunk_rows):
            r1 = min(n, r0 + chunk_rows)
            mu = np.exp(X[r0:r1] @ B.T + gamma0[r0:r1] @ Z.T + U[r0:r1] @ V.T)
            if family == "negbin":
                Y[r0:r1] = yr.negative_binomial(alpha, alpha / (alpha + mu))
            else:
                Y[r0:r1] = yr.poisson(mu)
    else:
        # large matrices: row chunks of `chunk_rows`, chunk k drawn from its own
        # PCG64 stream seeded with (seed + 11, k)
        _parallel_counts(Y, dict(X=X, B=B, G=gamma0, Z=Z, U=U, V=V, seed=seed + 11,
                                 family=family, alpha=alpha), chunk_rows)
    B0, A0, U0, V0 = _start_values(_rng(seed + 2000), Y, X, Z, d, "poisson")
    return Problem(family, "log", n, m, d, 3, 1, R, S, Y, X, Z, B0, A0, U0, V0,
                   nb_alpha=alpha, sched_seed=seed + 1000,
                   name=f"{family}_{n}x{m}_d{d}",
                   true=dict(B=B, A=gamma0, U=U, V=V, shift=c))


def gen_gaussian_lowrank(n=60, m=40, d=3, R=1, S=1, sing=(9.0, 6.0, 4.0),
                         noise=0.05, seed=1010):
    """Real matrix M + noise with planted singular values ``sing``, no covariates.

    p = q = 0, so the linear predictor is U V^T alone and the model reduces to
    a penalised rank-d factorisation of Y.
    """
    rng = _rng(seed)
    Qu, _ = np.linalg.qr(rng.normal(size=(n, d)))
    Qv, _ = np.linalg.qr(rng.normal(size=(m, d)))
    M = (Qu * np.asarray(sing[:d])) @ Qv.T
    Y = _f32(M + noise * rng.normal(size=(n, m)))
    r2 = _rng(seed + 2000)
    U0 = _f32(r2.normal(0.0, 0.3, size=(n, d)))
    V0 = _f32(r2.normal(0.0, 0.3, size=(m, d)))
    return Problem("gaussian", "identity", n, m, d, 0, 0, R, S, Y,
                   np.zeros((n, 0)), np.zeros((m, 0)), np.zeros((m, 0)),
                   np.zeros((n, 0)), U0, V0, sched_seed=seed + 1000,
                   name=f"gauss_{n}x{m}_d{d}", true=dict(M=M))


def gen_tiny(family="poisson", n=6, m=5, d=2, p=2, q=1, R=1, S=1, seed=1020,
             weights=False):
    """Tiny problem with general covariates for finite-difference checks.
    Families: poisson, negbin (alpha 5), gaussian (identity link, noise sd
    0.3, phi 0.7 in the fit), gamma (log link, shape 2: phi 0.5), invgauss
    (log link, shape 1/0.3: phi 0.3), bernoulli (logit link)."""
    rng = _rng(seed)
    X = _f32(np.column_stack([np.ones(n)] + [rng.normal(size=n) for _ in range(p - 1)]))
    Z = _f32(np.column_stack([np.ones(m)] + [rng.normal(size=m) for _ in range(q - 1)]))
    B = rng.normal(0.0, 0.3, size=(m, p))
    A = rng.normal(0.0, 0.3, size=(n, q))
    U = rng.normal(0.0, 0.4, size=(n, d))
    V = rng.normal(0.0, 0.4, size=(m, d))
    eta = X @ B.T + A @ Z.T + U @ V.T
    phi = 1.0
    if family == "gaussian":
        Y = _f32(eta + 0.3 * rng.normal(size=(n, m)))
        link, phi = "identity", 0.7
    elif family == "negbin":
        mu = np.exp(eta + 1.0)
        Y = rng.negative_binomial(5.0, 5.0 / (5.0 + mu)).astype(np.int32)
        link = "log"
    elif family == "gamma":
        phi = 0.5
        Y = _f32(rng.gamma(1.0 / phi, np.exp(eta) * phi))
        link = "log"
    elif family == "invgauss":
        phi = 0.3
        Y = _f32(rng.wald(np.exp(eta), 1.0 / phi))
        link = "log"
    elif family == "bernoulli":
        Y = (rng.random(size=(n, m)) < 1.0 / (1.0 + np.exp(-eta))).astype(np.int32)
        link = "logit"
    else:
        Y = rng.poisson(np.exp(eta + 1.0)).astype(np.int32)
        link = "log"
    W = _f32(rng.uniform(0.5, 2.0, size=(n, m))) if weights else None
    shift = 1.0 if family in ("poisson", "negbin") else 0.0
    true = dict(B=B, A=A, U=U, V=V, eta=eta + shift)
    return Problem(family, link, n, m, d, p, q, R, S, Y, X, Z, _f32(B), _f32(A),
                   _f32(U), _f32(V), phi=phi, W=W, sched_seed=seed + 1000,
                   true=true, name=f"tiny_{family}")


def holdout(Y, frac, seed):
    """Hide a uniformly drawn fraction of the entries (Section 5.2's protocol):
    returns (Y_train as float64 with NaN at the held-out entries, held-out
    mask)."""
    rng = _rng(seed)
    mask = rng.random(size=np.shape(Y)) < frac
    Yt = np.asarray(Y, np.float64).copy()
    Yt[mask] = np.nan
    return Yt, mask


# The workloads: shapes, families and seeds.  "c1".."c5" follow the order of
# the headline configurations (Poisson parity case, NB plain path, NB large
# BF16 path, batched fits, learned warm start).
CONFIGS = {
    "c1": dict(kind="poisson", n=1000, m=500, d=5, R=10, S=5, seed=1001),
    "c2": dict(kind="negbin", n=10_000, m=2_000, d=10, R=10, S=5, seed=1002,
               epochs=200),
    "c3": dict(kind="negbin", n=100_000, m=5_000, d=20, R=10, S=5, seed=1003),
}


def make_problem(name: str, **over) -> Problem:
    cfg = dict(CONFIGS[name])
    cfg.update(over)
    kind = cfg.pop("kind")
    cfg.pop("epochs", None)
    if kind == "poisson":
        return gen_poisson_small(**cfg)
    return gen_nb(**cfg)


def mlp_init(m, hidden, d, seed=4001):
    """Starting weights of the warm-start encoder (m -> hidden -> hidden -> d):
    each layer's weights and biases uniform on +-1/sqrt(fan_in), float32."""
    rng = _rng(seed)
    out = {}
    for name, (fo, fi) in (("1", (hidden, m)), ("2", (hidden, hidden)), ("3", (d, hidden))):
        lim = 1.0 / np.sqrt(fi)
        out["W" + name] = _f32(rng.uniform(-lim, lim, size=(fo, fi)))
        out["b" + name] = _f32(rng.uniform(-lim, lim, size=fo))
    return out


def gen_nb_rows(pr, n_new, seed=5005, chunk_rows=4096):
    """New rows for a problem from gen_nb: the same column side (B, Z, V and
    alpha of ``pr.true``) and fresh row draws (batch indicator, covariate,
    row intercept N(0, 0.5^2), scores N(0, 0.5^2)).  Returns (Y, X, U_true,
    gamma_true)."""
    rng = _rng(seed)
    d = pr.d
    batch = np.zeros(n_new)
    batch[rng.permutation(n_new)[: n_new // 2]] = 1.0
    X = _f32(np.column_stack([np.ones(n_new), batch, rng.normal(0.0, 1.0, size=n_new)]))
    gamma0 = rng.normal(0.0, 0.5, size=(n_new, 1))
    U = rng.normal(0.0, 0.5, size=(n_new, d))
    B, V = pr.true["B"], pr.true["V"]
    Y = np.empty((n_new, pr.m), dtype=np.int32)
    if n_new * pr.m < _PAR_THRESHOLD:
        yr = _rng(seed + 11)
        for r0 in range(0, n_new, chunk_rows):
            r1 = min(n_new, r0 + chunk_rows)
            mu = np.exp(X[r0:r1] @ B.T + gamma0[r0:r1] @ pr.Z.T + U[r0:r1] @ V.T)
            a = pr.nb_alpha
            Y[r0:r1] = yr.negative_binomial(a, a / (a + mu)) if pr.family == "negbin" else yr.poisson(mu)
    else:
        _parallel_counts(Y, dict(X=X, B=B, G=gamma0, Z=pr.Z, U=U, V=V, seed=seed + 11,
                                 family=pr.family, alpha=pr.nb_alpha), chunk_rows)
    return Y, X, U, gamma0
