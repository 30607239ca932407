"""Pins of the FP64 oracle against facts fixed outside it.

Each test ties a part of the oracle to something independent of its own code:
scipy's log-pmfs, finite differences, exact expectations over a support,
published RNG test vectors, closed-form minimisers (truncated / shrunken SVD)
and the invariants of the identifiability constraints.
"""
import copy
import os

import numpy as np
import pytest
from scipy import stats

from oracle import gmf_oracle as G
from synth import gen_gaussian_lowrank, gen_poisson_small, gen_tiny

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- families ---

def _loglik(family, y, mu, alpha=5.0, phi=1.0):
    if family == "poisson":
        return stats.poisson.logpmf(y, mu)
    if family == "negbin":
        return stats.nbinom.logpmf(y, alpha, alpha / (alpha + mu))
    if family == "gaussian":
        return stats.norm.logpdf(y, mu, np.sqrt(phi))
    raise ValueError


@pytest.mark.parametrize("family", ["poisson", "negbin"])
def test_unit_deviance_matches_scipy_logpmf(family):
    y = np.array([0, 0, 1, 2, 3, 7, 15, 40, 120])
    mu = np.array([0.01, 2.5, 0.3, 2.0, 5.5, 7.0, 3.0, 55.0, 100.0])
    ref = 2.0 * (_loglik(family, y, np.maximum(y, 1e-300)) - _loglik(family, y, mu))
    # the saturated model at y = 0 has log f(0, 0) = 0
    ref = np.where(y == 0, -2.0 * _loglik(family, y, mu), ref)
    got = G.unit_deviance(family, y, mu, 5.0)
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-12)


def test_gaussian_deviance_is_twice_negloglik_ratio():
    y = np.array([-1.3, 0.0, 2.2])
    mu = np.array([0.5, -0.7, 2.0])
    ref = 2.0 * (_loglik("gaussian", y, y) - _loglik("gaussian", y, mu))
    np.testing.assert_allclose(G.unit_deviance("gaussian", y, mu), ref, rtol=1e-12)


def test_deviance_special_values():
    mu = np.array([0.1, 1.0, 7.5])
    np.testing.assert_allclose(G.unit_deviance("poisson", 0 * mu, mu), 2 * mu)
    for fam in ("poisson", "negbin", "gaussian"):
        y = np.array([1.0, 3.0, 8.0])
        np.testing.assert_allclose(G.unit_deviance(fam, y, y), 0.0, atol=1e-14)
    # NB tends to Poisson as alpha -> infinity
    y = np.array([0.0, 2.0, 9.0])
    np.testing.assert_allclose(G.unit_deviance("negbin", y, mu, 1e9),
                               G.unit_deviance("poisson", y, mu), rtol=1e-6, atol=1e-8)


def _nll_entry(family, link, y, eta, w, phi, alpha):
    mu = G.inverse_link(link, eta, 1e-300, 700.0)
    return w * G.unit_deviance(family, y, mu, alpha) / (2.0 * phi)


@pytest.mark.parametrize("family,link", [("poisson", "log"), ("negbin", "log"),
                                         ("gaussian", "identity")])
def test_first_derivative_is_fd_of_nll(family, link):
    rng = np.random.default_rng(5)
    eta = rng.normal(0.3, 0.8, size=40)
    y = (rng.poisson(2.0, size=40) if family != "gaussian" else rng.normal(size=40))
    w = rng.uniform(0.5, 2.0, size=40)
    phi = 1.0 if family != "gaussian" else 0.6
    mu = G.inverse_link(link, eta)
    D1, _ = G.deviance_derivatives(family, link, y, mu, w, phi, 5.0)
    h = 1e-6
    fd = (_nll_entry(family, link, y, eta + h, w, phi, 5.0)
          - _nll_entry(family, link, y, eta - h, w, phi, 5.0)) / (2 * h)
    np.testing.assert_allclose(D1, fd, rtol=1e-7, atol=1e-9)


@pytest.mark.parametrize("family", ["poisson", "negbin"])
def test_fisher_weight_is_expected_second_derivative(family):
    """D2 = E_y[d^2 NLL / d eta^2], summed exactly over the support."""
    alpha = 5.0
    for eta in (-1.5, 0.2, 1.7):
        mu = np.exp(eta)
        ys = np.arange(0, 400)
        pmf = np.exp(_loglik(family, ys, mu, alpha))
        assert pmf.sum() > 1 - 1e-13
        h = 1e-4
        sec = (_nll_entry(family, "log", ys, eta + h, 1.0, 1.0, alpha)
               - 2 * _nll_entry(family, "log", ys, eta, 1.0, 1.0, alpha)
               + _nll_entry(family, "log", ys, eta - h, 1.0, 1.0, alpha)) / h ** 2
        _, D2 = G.deviance_derivatives(family, "log", ys[:1], np.array([mu]), None,
                                       1.0, alpha)
        np.testing.assert_allclose(np.sum(pmf * sec), D2[0], rtol=1e-6)


def test_nb_observed_is_fisher_times_alpha_mu():
    """Observed second derivative = Fisher weight * alpha(mu) (Section 3)."""
    a = 5.0
    for y, eta in [(0, 0.3), (4, -0.2), (11, 1.9)]:
        mu = np.exp(eta)
        h = 1e-4
        sec = (_nll_entry("negbin", "log", y, eta + h, 1.0, 1.0, a)
               - 2 * _nll_entry("negbin", "log", y, eta, 1.0, 1.0, a)
               + _nll_entry("negbin", "log", y, eta - h, 1.0, 1.0, a)) / h ** 2
        nu = mu * (1 + mu / a)
        dnu = 1 + 2 * mu / a
        gp, gpp = 1 / mu, -1 / mu ** 2
        alpha_mu = 1 + (y - mu) * (dnu / nu + gpp / gp)
        _, D2 = G.deviance_derivatives("negbin", "log", y, np.array([mu]), None, 1.0, a)
        np.testing.assert_allclose(sec, D2[0] * alpha_mu, rtol=1e-5)


# ------------------------------------------------------------- schedule ---

def test_splitmix64_published_vector():
    lines = [ln.split("#")[0].strip() for ln in
             open(os.path.join(GOLDEN, "splitmix64_vectors.txt"))]
    lines = [ln for ln in lines if ln]
    seed = int(lines[0].split()[1])
    want = [int(x) for x in lines[1:]]
    got = [G.splitmix_draw(seed, k) for k in range(len(want))]
    assert got == want


def test_partitions_are_bijections_and_sweeps_cover_columns():
    perm = G.permutation(77, G.STREAM_ROWS, 1003)
    assert sorted(perm.tolist()) == list(range(1003))
    blocks = G.partition(perm, 10)
    assert sum(len(b) for b in blocks) == 1003
    assert max(len(b) for b in blocks) - min(len(b) for b in blocks) <= 1
    assert sorted(np.concatenate(blocks).tolist()) == list(range(1003))
    S = 5
    for sweep in range(4):
        seen = [G.col_block_of_step(sweep * S + k + 1, S) for k in range(S)]
        assert seen == list(range(S))


def test_row_draws_are_uniform():
    R = 10
    draws = np.array([G.row_block_draw(123, t, R) for t in range(1, 20001)])
    counts = np.bincount(draws, minlength=R)
    chi2 = ((counts - 2000.0) ** 2 / 2000.0).sum()
    assert chi2 < stats.chi2.ppf(0.999, R - 1)


def test_uniform_below_is_floor_of_scaled_draw():
    for u in (0, 1, 2 ** 63, 2 ** 64 - 1, 0x123456789ABCDEF0):
        for n in (1, 7, 10, 100003):
            assert G.uniform_below(u, n) == int(np.floor(u / 2.0 ** 64 * n)) or \
                abs(u / 2.0 ** 64 * n - round(u / 2.0 ** 64 * n)) < 1e-9


# --------------------------------------------------------------- gradients --

def _oracle(pr, **over):
    kw = dict(family=pr.family, link=pr.link, phi=pr.phi, nb_alpha=pr.nb_alpha,
              R=pr.R, S=pr.S, seed=pr.sched_seed)
    kw.update(over)
    cfg = G.Config(**kw)
    return G.OracleGMF(cfg, pr.Y, pr.X, pr.Z, pr.B0, pr.A0, pr.U0, pr.V0, W=pr.W)


def _fd_grad(o, h=1e-6):
    """Central finite differences of the penalised objective in (Gamma,U) and (B,V)."""
    g_row = np.zeros((o.n, o.q + o.d))
    g_col = np.zeros((o.m, o.p + o.d))
    for arrname, gout, offset in (("A", g_row, 0), ("U", g_row, o.q),
                                  ("B", g_col, 0), ("V", g_col, o.p)):
        arr = getattr(o, arrname)
        for idx in np.ndindex(arr.shape):
            old = arr[idx]
            arr[idx] = old + h
            fp = o.objective()
            arr[idx] = old - h
            fm = o.objective()
            arr[idx] = old
            gout[idx[0], offset + idx[1]] = (fp - fm) / (2 * h)
    return g_row, g_col


@pytest.mark.parametrize("family,weights", [("poisson", False), ("negbin", True),
                                            ("gaussian", True)])
def test_full_batch_gradient_equals_fd_gradient(family, weights):
    pr = gen_tiny(family, weights=weights)
    o = _oracle(pr, alpha1=1.0, alpha2=1.0, lam=(0.3, 0.2, 0.7, 0.5))
    g_row_fd, g_col_fd = _fd_grad(o)
    g_row, g_col = o.full_gradient()
    np.testing.assert_allclose(g_row, g_row_fd, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(g_col, g_col_fd, rtol=1e-6, atol=1e-7)
    # with R = S = 1 and alpha1 = 1 the smoothed gradient after one step is
    # the minibatch gradient of the whole matrix, i.e. the exact gradient
    o.step()
    np.testing.assert_allclose(o.Grow, g_row_fd, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(o.Gcol, g_col_fd, rtol=1e-6, atol=1e-7)


def test_poisson_hessian_diagonal_is_fd_second_derivative():
    """For the canonical Poisson-log pair the Fisher diagonal is the exact one."""
    pr = gen_tiny("poisson")
    o = _oracle(pr, alpha1=1.0, alpha2=1.0, lam=(0.0, 0.0, 0.4, 0.4))
    base = copy.deepcopy(o)
    o.step()
    h = 1e-4
    for arrname, H, col in (("U", o.Hrow, base.q), ("V", o.Hcol, base.p),
                            ("A", o.Hrow, 0), ("B", o.Hcol, 0)):
        arr = getattr(base, arrname)
        for idx in [(0, 0), (2, arr.shape[1] - 1), (arr.shape[0] - 1, 0)]:
            old = arr[idx]
            f0 = base.objective()
            arr[idx] = old + h
            fp = base.objective()
            arr[idx] = old - h
            fm = base.objective()
            arr[idx] = old
            np.testing.assert_allclose(H[idx[0], col + idx[1]], (fp - 2 * f0 + fm) / h ** 2,
                                       rtol=1e-5)


def test_minibatch_gradients_average_to_full_gradient():
    """Averaging over equal-size blocks recovers the full gradient (eq. 15)."""
    pr = gen_tiny("negbin", n=12, m=10, R=3, S=2)
    pr.R, pr.S = 3, 2
    o = _oracle(pr, alpha1=1.0, alpha2=1.0, lam=(0.1, 0.2, 0.3, 0.4), R=3, S=2,
                rate0=1e-300)
    g_row, g_col = o.full_gradient()
    row_sum = np.zeros_like(g_row)
    col_sum = np.zeros_like(g_col)
    for r in range(3):
        for s in range(2):
            c = copy.deepcopy(o)
            c.step_block(1, r, s)
            I, J = c.row_blocks[r], c.col_blocks[s]
            row_sum[I] += c.Grow[I]
            col_sum[J] += c.Gcol[J]
    # each row block is paired with S column blocks and vice versa
    np.testing.assert_allclose(row_sum / 2, g_row, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(col_sum / 3, g_col, rtol=1e-11, atol=1e-12)


def test_bias_corrected_direction_is_newton_direction_for_constant_inputs():
    """Fed the same minibatch gradient every step, the bias-corrected direction
    alpha_t Gbar_t / Hbar_t equals G_hat / H_hat at every t (eq. 11-12)."""
    pr = gen_tiny("poisson")
    o = _oracle(pr, damping=0.0, rate0=0.7, decay=0.3)
    ref = copy.deepcopy(o)
    ref.cfg = G.Config(**{**o.cfg.__dict__, "alpha1": 1.0, "alpha2": 1.0})
    ref.step()
    newton_row = ref.Grow / ref.Hrow
    newton_col = ref.Gcol / ref.Hcol
    for t in range(1, 40):
        saved = o.params()
        o.step()
        rho = G.learning_rate(o.cfg, t)
        np.testing.assert_allclose((np.hstack([saved[1], saved[2]])
                                    - np.hstack([o.A, o.U])) / rho, newton_row, rtol=1e-9)
        np.testing.assert_allclose((np.hstack([saved[0], saved[3]])
                                    - np.hstack([o.B, o.V])) / rho, newton_col, rtol=1e-9)
        o.B, o.A, o.U, o.V = saved


def test_quasi_newton_special_case_and_monotone_decrease():
    """R=S=1, alpha1=alpha2=1, delta=0 is the diagonal quasi-Newton of eq. 10."""
    pr = gen_tiny("poisson", n=8, m=7)
    o = _oracle(pr, alpha1=1.0, alpha2=1.0, damping=0.0, rate0=0.2, decay=0.0,
                lam=(0.0, 0.0, 0.5, 0.5))
    f_prev = o.objective()
    for _ in range(200):
        g_row, g_col = o.full_gradient()
        before_u = o.U.copy()
        o.step()
        # the U update equals -rho * G/H with G the exact gradient
        H_u = o.Hrow[:, o.q:]
        np.testing.assert_allclose(o.U, before_u - 0.2 * g_row[:, o.q:] / H_u,
                                   rtol=1e-10, atol=1e-12)
        f = o.objective()
        assert f <= f_prev * (1 + 1e-12)
        f_prev = f


@pytest.mark.parametrize("lam", [0.0, 0.5])
def test_gaussian_full_batch_reaches_truncated_svd(lam):
    """Gaussian-identity without covariates: the minimiser of eq. 6 is the
    rank-d SVD of Y with singular values shrunk to (s_k - lambda)_+."""
    pr = gen_gaussian_lowrank()
    o = _oracle(pr, lam=(0.0, 0.0, lam, lam), rate0=0.5, decay=0.0, alpha1=1.0,
                alpha2=1.0, damping=0.0)
    o.steps(1500)
    P, s, Qt = np.linalg.svd(pr.Y, full_matrices=False)
    d = pr.d
    M = (P[:, :d] * np.maximum(s[:d] - lam, 0)) @ Qt[:d]
    err = np.linalg.norm(o.U @ o.V.T - M) / np.linalg.norm(M)
    assert err < 1e-6


def test_sgd_converges_to_stationary_point_full_batch():
    from scipy.optimize import minimize
    pr = gen_tiny("poisson", n=7, m=6)
    o = _oracle(pr, alpha1=1.0, alpha2=1.0, damping=0.0, rate0=0.3, decay=0.0,
                lam=(0.1, 0.1, 0.5, 0.5))
    o.steps(15000)
    g_row, g_col = o.full_gradient()
    gnorm = np.sqrt((g_row ** 2).sum() + (g_col ** 2).sum())
    assert gnorm < 1e-8 * max(1.0, abs(o.objective()))
    # an independent optimiser from the same start reaches the same objective
    o2 = _oracle(pr, lam=(0.1, 0.1, 0.5, 0.5))
    shapes = [o2.B.shape, o2.A.shape, o2.U.shape, o2.V.shape]

    def unpack(x):
        out, k = [], 0
        for sh in shapes:
            sz = int(np.prod(sh))
            out.append(x[k:k + sz].reshape(sh))
            k += sz
        return out

    def f(x):
        o2.B, o2.A, o2.U, o2.V = unpack(x)
        gr, gc = o2.full_gradient()
        gB, gV = gc[:, :o2.p], gc[:, o2.p:]
        gA, gU = gr[:, :o2.q], gr[:, o2.q:]
        return o2.objective(), np.concatenate([gB.ravel(), gA.ravel(), gU.ravel(),
                                               gV.ravel()])

    x0 = np.concatenate([pr.B0.ravel(), pr.A0.ravel(), pr.U0.ravel(), pr.V0.ravel()])
    res = minimize(f, x0, jac=True, method="L-BFGS-B",
                   options=dict(maxiter=20000, ftol=1e-15, gtol=1e-12))
    assert abs(res.fun - o.objective()) <= 1e-8 * abs(o.objective())


# --------------------------------------------------------- post-processing --

def _pp_inputs(seed=3):
    rng = np.random.default_rng(seed)
    n, m, p, q, d = 30, 20, 3, 2, 4
    X = np.column_stack([np.ones(n), rng.normal(size=(n, p - 1))])
    Z = np.column_stack([np.ones(m), rng.normal(size=(m, q - 1))])
    B = rng.normal(size=(m, p))
    A = rng.normal(size=(n, q))
    U = rng.normal(size=(n, d))
    V = rng.normal(size=(m, d))
    return X, Z, B, A, U, V


def test_postprocess_invariants():
    X, Z, B, A, U, V = _pp_inputs()
    eta = X @ B.T + A @ Z.T + U @ V.T
    B2, A2, U2, V2 = G.postprocess_A_B1(X, Z, B, A, U, V)
    np.testing.assert_allclose(X @ B2.T + A2 @ Z.T + U2 @ V2.T, eta, atol=1e-12)
    for M in (X.T @ A2, X.T @ U2, Z.T @ V2):
        assert np.abs(M).max() < 1e-12
    np.testing.assert_allclose(V2.T @ V2, np.eye(U.shape[1]), atol=1e-12)
    UtU = U2.T @ U2
    off = UtU - np.diag(np.diag(UtU))
    assert np.abs(off).max() < 1e-10
    assert np.all(np.diff(np.diag(UtU)) <= 0)
    for k in range(V2.shape[1]):
        assert V2[np.nonzero(V2[:, k])[0][0], k] > 0


def test_postprocess_is_rotation_invariant():
    """Lemma 2: (U Q, V Q) for orthogonal Q yields the same constrained output."""
    X, Z, B, A, U, V = _pp_inputs(4)
    Q, _ = np.linalg.qr(np.random.default_rng(9).normal(size=(U.shape[1],) * 2))
    out1 = G.postprocess_A_B1(X, Z, B, A, U, V)
    out2 = G.postprocess_A_B1(X, Z, B, A, U @ Q, V @ Q)
    for a, b in zip(out1, out2):
        np.testing.assert_allclose(a, b, atol=1e-10)


# -------------------------------------------------------------- projection --

def test_projection_rows_are_independent_and_reach_row_optimum():
    pr = gen_poisson_small(n=60, m=40, d=3, R=2, S=2)
    cfg = G.Config(family="poisson", link="log", R=2, S=2, seed=pr.sched_seed,
                   rate0=0.3, decay=0.0, lam=(0, 0, 0.5, 0.5))
    cols = G.partition(G.permutation(cfg.seed, G.STREAM_COLS, pr.m), 2)
    B, V = pr.true["B"], pr.true["V"]
    A0 = np.zeros((pr.n, 1))
    U0 = np.zeros((pr.n, pr.d))
    A, U = G.project_rows(cfg, pr.Y, pr.X, pr.Z, B, V, A0, U0, 60, cols)
    sub = np.arange(5, 25)
    As, Us = G.project_rows(cfg, pr.Y[sub], pr.X[sub], pr.Z, B, V, A0[sub], U0[sub], 60, cols)
    np.testing.assert_allclose(As, A[sub], rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(Us, U[sub], rtol=1e-13, atol=1e-14)
    # with the full column set (S = 1) the iteration reaches each row's
    # optimum: minimise that row's deviance/2 + penalty directly
    from scipy.optimize import minimize
    A, U = G.project_rows(cfg, pr.Y, pr.X, pr.Z, B, V, A0, U0, 400, [np.arange(pr.m)])
    i = 3

    def f(x):
        eta = pr.X[i] @ B.T + x[0] * pr.Z[:, 0] + V @ x[1:]
        mu = np.exp(eta)
        return 0.5 * G.unit_deviance("poisson", pr.Y[i], mu).sum() + 0.25 * np.sum(x[1:] ** 2)

    res = minimize(f, np.zeros(1 + pr.d), method="BFGS", options=dict(gtol=1e-10))
    np.testing.assert_allclose(np.concatenate([A[i], U[i]]), res.x, atol=1e-6)


# ------------------------------------------------- projection start values --

def test_row_intercept_start_matches_row_totals():
    """With U = 0 the log-link intercept makes each row's fitted total equal
    its count total + 1/2; the identity-link intercept makes the mean residual
    zero (both by construction of the definition, checked from the mean)."""
    rng = np.random.default_rng(11)
    n, m, p = 9, 13, 2
    X = np.column_stack([np.ones(n), rng.normal(size=n)])
    B = rng.normal(0, 0.4, size=(m, p))
    Y = rng.poisson(2.0, size=(n, m))
    Y[3] = 0                                  # an all-zero row
    cfg = G.Config(family="poisson")
    A0 = G.row_intercept_start(cfg, Y, X, B, q=2)
    mu = np.exp(X @ B.T + A0[:, :1])
    np.testing.assert_allclose(mu.sum(axis=1), Y.sum(axis=1) + 0.5, rtol=1e-12)
    assert np.all(A0[:, 1] == 0)
    cfg_g = G.Config(family="gaussian", link="identity")
    Yg = rng.normal(size=(n, m))
    Ag = G.row_intercept_start(cfg_g, Yg, X, B, q=1)
    np.testing.assert_allclose((Yg - X @ B.T - Ag).mean(axis=1), 0.0, atol=1e-12)


def test_warm_start_rows_picks_lower_row_deviance():
    """Brute force: per row, sum the unit deviances entry by entry for both
    candidates and compare with the selection."""
    rng = np.random.default_rng(12)
    n, m, p, q, d = 8, 10, 1, 1, 2
    X = np.ones((n, p))
    Z = np.ones((m, q))
    B = rng.normal(0, 0.3, size=(m, p))
    V = rng.normal(0, 0.5, size=(m, d))
    U_true = rng.normal(0, 0.8, size=(n, d))
    Y = rng.poisson(np.exp(X @ B.T + U_true @ V.T))
    cand = U_true.copy()
    cand[::2] = -3.0 * U_true[::2]             # poor candidates on even rows
    cfg = G.Config(family="poisson")
    A0 = G.row_intercept_start(cfg, Y, X, B, q)
    U0, warm, dc, d0 = G.warm_start_rows(cfg, Y, X, Z, B, V, A0, cand)
    for i in range(n):
        def dev(u):
            tot = 0.0
            for j in range(m):
                eta = X[i] @ B[j] + A0[i] @ Z[j] + u @ V[j]
                tot += float(G.unit_deviance("poisson", Y[i, j], np.exp(eta)))
            return tot
        a, b = dev(cand[i]), dev(np.zeros(d))
        assert abs(a - dc[i]) <= 1e-10 * max(1.0, a) and abs(b - d0[i]) <= 1e-10 * max(1.0, b)
        assert warm[i] == (a < b)
        np.testing.assert_array_equal(U0[i], cand[i] if a < b else np.zeros(d))
    assert warm.any() and (~warm).any()       # both outcomes occur


# ------------------------------------------------ step sizes (Section 3.2) --

def _rate_table():
    rows = []
    for ln in open(os.path.join(GOLDEN, "learning_rate_table.txt")):
        ln = ln.split("#")[0].split()
        if ln:
            rows.append((float(ln[0]), float(ln[1]), float(ln[2]), int(ln[3]), float(ln[4])))
    return rows


def test_learning_rate_matches_hand_table():
    """rho_t against values of the definition evaluated outside the oracle
    (30-digit decimal arithmetic), at t = 1, 2, 50, 1000 with k1 != 0: a shift
    of t, or k0, k1 or tau misplaced, moves at least one entry."""
    rows = _rate_table()
    assert len(rows) == 8
    for k0, k1, tau, t, want in rows:
        cfg = G.Config(rate0=k0, decay=k1, tau=tau)
        assert abs(G.learning_rate(cfg, t) - want) <= 1e-14 * want


def test_step_uses_rate_of_global_counter():
    """The displacement of step t divided by the Newton direction G/H is
    rho_t of the hand table (alpha1 = alpha2 = 1, damping 0, full batch): the
    oracle's step applies the rate of its own global counter t = 1, 2, ...."""
    k0, k1, tau = 0.05, 0.05, 0.75
    want = {t: v for a, b, c, t, v in _rate_table() if (a, b, c) == (k0, k1, tau)}
    pr = gen_tiny("poisson")
    o = _oracle(pr, alpha1=1.0, alpha2=1.0, damping=0.0, rate0=k0, decay=k1, tau=tau)
    for t in range(1, 1001):
        if t in want:
            before = np.hstack([o.A, o.U])
            o.step()
            disp = (before - np.hstack([o.A, o.U])) / (o.Grow / o.Hrow)
            np.testing.assert_allclose(disp, want[t], rtol=1e-8)
        else:
            o.step()
        assert o.t == t


# --------------------------------------- Fisher weight with w and phi ------

@pytest.mark.parametrize("w,phi", [(1.0, 1.0), (2.5, 1.0), (1.0, 0.4), (0.3, 3.0)])
def test_gaussian_d2_with_weights_and_dispersion_is_fd_second_derivative(w, phi):
    """Gaussian-identity: the per-entry NLL w (y - mu)^2 / (2 phi) has second
    derivative w / phi in eta (canonical link: observed = Fisher).  Central
    second differences of the NLL pin D2 including its w and phi factors."""
    rng = np.random.default_rng(21)
    y = rng.normal(size=12)
    eta = rng.normal(size=12)
    h = 1e-3
    sec = (_nll_entry("gaussian", "identity", y, eta + h, w, phi, 5.0)
           - 2 * _nll_entry("gaussian", "identity", y, eta, w, phi, 5.0)
           + _nll_entry("gaussian", "identity", y, eta - h, w, phi, 5.0)) / h ** 2
    wv = np.full(12, w)
    _, D2 = G.deviance_derivatives("gaussian", "identity", y, eta, wv, phi, 5.0)
    np.testing.assert_allclose(D2, sec, rtol=1e-6)
    np.testing.assert_allclose(D2, w / phi, rtol=1e-14)


@pytest.mark.parametrize("family", ["poisson", "negbin"])
@pytest.mark.parametrize("w,phi", [(2.5, 1.0), (0.4, 1.7)])
def test_fisher_weight_with_weights_and_dispersion(family, w, phi):
    """D2 = E_y[d^2 (w D / (2 phi)) / d eta^2] for weighted entries with a
    dispersion, summed exactly over the support of the unweighted law."""
    alpha = 5.0
    for eta in (-0.7, 1.1):
        mu = np.exp(eta)
        ys = np.arange(0, 400)
        pmf = np.exp(_loglik(family, ys, mu, alpha))
        h = 1e-4
        sec = (_nll_entry(family, "log", ys, eta + h, w, phi, alpha)
               - 2 * _nll_entry(family, "log", ys, eta, w, phi, alpha)
               + _nll_entry(family, "log", ys, eta - h, w, phi, alpha)) / h ** 2
        _, D2 = G.deviance_derivatives(family, "log", ys[:1], np.array([mu]),
                                       np.array([w]), phi, alpha)
        np.testing.assert_allclose(np.sum(pmf * sec), D2[0], rtol=1e-6)


# ------------------------------------------- Fisher-Yates uniformity -------

@pytest.mark.parametrize("n", [3, 4])
def test_permutation_is_uniform_over_all_orderings(n):
    """Over many stream keys every one of the n! orderings appears equally
    often (chi-square at 0.999).  A shuffle drawing j from [0, i) (Sattolo:
    cyclic permutations only) or from [0, n) (biased) fails."""
    from itertools import permutations
    from math import factorial
    index = {p: k for k, p in enumerate(permutations(range(n)))}
    nperm = factorial(n)
    draws = 1000 * nperm
    counts = np.zeros(nperm)
    for seed in range(draws):
        counts[index[tuple(G.permutation(seed, G.STREAM_ROWS, n).tolist())]] += 1
    expect = draws / nperm
    chi2 = ((counts - expect) ** 2 / expect).sum()
    assert counts.min() > 0
    assert chi2 < stats.chi2.ppf(0.999, nperm - 1)


def test_permutation_positions_are_uniform_for_larger_n():
    """Each element lands in each position with probability 1/n (n = 10)."""
    n, draws = 10, 20000
    pos = np.zeros((n, n))
    for seed in range(draws):
        perm = G.permutation(seed, G.STREAM_COLS, n)
        pos[np.arange(n), perm] += 1
    expect = draws / n
    chi2 = ((pos - expect) ** 2 / expect).sum()
    assert chi2 < stats.chi2.ppf(0.999, (n - 1) * (n - 1))
