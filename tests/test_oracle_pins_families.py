"""Pins of the oracle's Gamma, inverse-Gaussian and Bernoulli families, the
missing-value imputation, per-column NB shapes, the stochastic dispersion and
NB-shape estimators and the out-of-sample metrics, against what the
mathematics fixes: scipy log-densities, finite differences of the per-entry
NLL, the expectation of the second derivative, finite-difference gradients of
the objective over the observed entries, the consistency of the estimators on
data drawn with known dispersion, and the special cases of the metrics."""
import copy

import numpy as np
import pytest
from scipy import stats

from oracle import gmf_oracle as G
from synth import gen_tiny, holdout


def _oracle(pr, Y=None, **over):
    kw = dict(family=pr.family, link=pr.link, phi=pr.phi, nb_alpha=pr.nb_alpha,
              R=pr.R, S=pr.S, seed=pr.sched_seed)
    kw.update(over)
    return G.OracleGMF(G.Config(**kw), pr.Y if Y is None else Y, pr.X, pr.Z, pr.B0, pr.A0,
                       pr.U0, pr.V0, W=pr.W)


def test_new_unit_deviances_match_scipy_logdensities():
    y = np.array([0.2, 1.0, 3.5, 0.05])
    mu = np.array([0.7, 1.0, 2.0, 0.3])
    phi = 0.4
    # Gamma(mean mu, dispersion phi): shape 1/phi, scale mu phi
    lg = lambda m: stats.gamma.logpdf(y, a=1.0 / phi, scale=m * phi)
    np.testing.assert_allclose(G.unit_deviance("gamma", y, mu), 2 * phi * (lg(y) - lg(mu)),
                               rtol=1e-10)
    # inverse Gaussian(mean mu, shape lambda = 1/phi): scipy invgauss(mu/lambda, scale=lambda)
    lam = 1.0 / phi
    li = lambda m: stats.invgauss.logpdf(y, m / lam, scale=lam)
    np.testing.assert_allclose(G.unit_deviance("invgauss", y, mu), 2 * phi * (li(y) - li(mu)),
                               rtol=1e-10)
    yb = np.array([0.0, 1.0, 1.0, 0.0])
    mb = np.array([0.2, 0.9, 0.35, 0.6])
    np.testing.assert_allclose(G.unit_deviance("bernoulli", yb, mb),
                               -2 * stats.bernoulli.logpmf(yb, mb), rtol=1e-12)
    assert np.allclose(G.unit_deviance("gamma", y, y), 0) and np.allclose(
        G.unit_deviance("invgauss", y, y), 0)


def _nll(family, link, y, eta, w, phi, alpha=5.0):
    mu = G.inverse_link(link, eta, 1e-300, 700.0)
    return w * G.unit_deviance(family, y, mu, alpha) / (2.0 * phi)


@pytest.mark.parametrize("family,link", [("gamma", "log"), ("invgauss", "log"),
                                         ("bernoulli", "logit")])
def test_first_derivative_is_fd_of_nll_new_families(family, link):
    rng = np.random.default_rng(11)
    eta = rng.normal(0.1, 0.7, size=30)
    y = rng.integers(0, 2, 30).astype(float) if family == "bernoulli" else rng.gamma(2.0, 0.7, 30)
    w = rng.uniform(0.5, 2.0, 30)
    phi = 0.6
    mu = G.inverse_link(link, eta)
    D1, _ = G.deviance_derivatives(family, link, y, mu, w, phi)
    h = 1e-6
    fd = (_nll(family, link, y, eta + h, w, phi) - _nll(family, link, y, eta - h, w, phi)) / (2 * h)
    np.testing.assert_allclose(D1, fd, rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("family,link", [("gamma", "log"), ("invgauss", "log")])
def test_fisher_weight_new_families_is_expected_second_derivative(family, link):
    """For these families the second derivative of the NLL in eta is affine in
    y, so its expectation is its value at y = E[y] = mu."""
    w, phi = 1.7, 0.45
    for eta in (-0.8, 0.3, 1.2):
        mu = np.exp(eta)
        h = 1e-4
        sec = lambda yy: (_nll(family, link, yy, eta + h, w, phi)
                          - 2 * _nll(family, link, yy, eta, w, phi)
                          + _nll(family, link, yy, eta - h, w, phi)) / h ** 2
        # affine in y: the midpoint of two values is the value at the midpoint
        np.testing.assert_allclose(0.5 * (sec(0.5 * mu) + sec(1.5 * mu)), sec(mu), rtol=1e-5)
        _, D2 = G.deviance_derivatives(family, link, np.array([mu]), np.array([mu]), w, phi)
        np.testing.assert_allclose(D2[0], sec(mu), rtol=1e-5)


def test_bernoulli_fisher_weight_is_expected_second_derivative():
    w, phi = 0.8, 1.0
    for eta in (-2.0, 0.1, 1.4):
        mu = 1 / (1 + np.exp(-eta))
        h = 1e-4
        sec = lambda yy: (_nll("bernoulli", "logit", yy, eta + h, w, phi)
                          - 2 * _nll("bernoulli", "logit", yy, eta, w, phi)
                          + _nll("bernoulli", "logit", yy, eta - h, w, phi)) / h ** 2
        expect = (1 - mu) * sec(0.0) + mu * sec(1.0)
        _, D2 = G.deviance_derivatives("bernoulli", "logit", np.array([1.0]), np.array([mu]),
                                       w, phi)
        np.testing.assert_allclose(D2[0], expect, rtol=1e-5)


def _fd_grad(o, h=1e-6):
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


@pytest.mark.parametrize("family", ["poisson", "negbin", "gaussian", "gamma", "invgauss",
                                    "bernoulli"])
def test_full_batch_gradient_with_missing_entries_is_fd_of_observed_objective(family):
    """Imputing y <- mu makes the missing entries' D1 zero: the full-batch
    gradient is the gradient of the objective summed over the observed
    entries only."""
    pr = gen_tiny(family, n=7, m=6, weights=family in ("negbin", "gamma"))
    Yt, mask = holdout(pr.Y, 0.3, seed=5)
    assert 0 < mask.sum() < mask.size
    o = _oracle(pr, Y=Yt, alpha1=1.0, alpha2=1.0, lam=(0.3, 0.2, 0.7, 0.5))
    g_row_fd, g_col_fd = _fd_grad(o)
    o.step()
    np.testing.assert_allclose(o.Grow, g_row_fd, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(o.Gcol, g_col_fd, rtol=1e-6, atol=1e-7)


def test_missing_entries_keep_their_fisher_weight():
    """The imputed entries keep the curvature D2 of their mean (the Fisher
    weight does not depend on y): the smoothed Hessians of one full-batch
    step are those of the complete matrix, while the gradients differ."""
    pr = gen_tiny("negbin", n=7, m=6)
    Yt, _ = holdout(pr.Y, 0.3, seed=6)
    a = _oracle(pr, alpha1=1.0, alpha2=1.0)
    b = _oracle(pr, Y=Yt, alpha1=1.0, alpha2=1.0)
    a.step()
    b.step()
    np.testing.assert_allclose(a.Hrow, b.Hrow, rtol=1e-13)
    np.testing.assert_allclose(a.Hcol, b.Hcol, rtol=1e-13)
    assert not np.allclose(a.Grow, b.Grow)


def test_per_column_nb_shape():
    pr = gen_tiny("negbin", n=9, m=8, R=1, S=2)
    alpha = np.full(pr.m, 5.0)
    a = _oracle(pr, R=1, S=2)
    b = _oracle(pr, R=1, S=2, nb_alpha=alpha)
    a.steps(4)
    b.steps(4)
    for x, y in ((a.U, b.U), (a.V, b.V), (a.B, b.B), (a.Hcol, b.Hcol)):
        assert np.array_equal(x, y)
    # with distinct shapes the full-batch gradient is the FD gradient
    alpha = np.linspace(0.5, 20.0, pr.m)
    o = _oracle(pr, R=1, S=1, nb_alpha=alpha, alpha1=1.0, alpha2=1.0, lam=(0.1, 0.1, 0.5, 0.5))
    g_row_fd, g_col_fd = _fd_grad(o)
    o.step()
    np.testing.assert_allclose(o.Grow, g_row_fd, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(o.Gcol, g_col_fd, rtol=1e-6, atol=1e-7)
    # the deviance uses each column's shape
    mu = G.inverse_link("log", o.eta_full())
    dev = sum(G.unit_deviance("negbin", o.Y[:, j], mu[:, j], alpha[j]).sum() for j in range(pr.m))
    np.testing.assert_allclose(o.full_deviance(), dev, rtol=1e-12)


def test_block_estimates_average_to_the_full_batch_estimates():
    """With rho_t = 1 each step's smoothed estimate is its block estimate; over
    the R x S equal blocks of one state the Pearson estimates average to the
    full-data Pearson estimate (the n m / (n* m*) scaling), which is the R = S
    = 1 estimate."""
    pr = gen_tiny("gamma", n=12, m=10, R=3, S=2)
    kw = dict(alpha1=1.0, alpha2=1.0, rate0=1.0, decay=0.0, tau=1.0, estimate_phi=True)
    vals = []
    for r in range(3):
        for s in range(2):
            o = _oracle(pr, R=3, S=2, **kw)
            o.step_block(1, r, s)
            vals.append(o.phi_bar)
    full = _oracle(pr, R=1, S=1, **kw)
    full.step()
    np.testing.assert_allclose(np.mean(vals), full.phi_bar, rtol=1e-12)


def test_dispersion_estimates_are_consistent():
    """On data drawn with known dispersion and at the true means, the Pearson
    estimate recovers phi (Gamma, phi = 0.5) and the moment estimate recovers
    the NB shape (alpha = 5), within Monte-Carlo error."""
    pr = gen_tiny("gamma", n=600, m=400, d=2, R=1, S=1, seed=77)
    t = pr.true
    o = G.OracleGMF(G.Config(family="gamma", link="log", phi=1.0, R=1, S=1, rate0=1.0,
                             decay=0.0, estimate_phi=True), pr.Y, pr.X, pr.Z, t["B"], t["A"],
                    t["U"], t["V"])
    o.step()
    N = o.n * o.m - o.m * o.p - o.n * o.q - (o.n + o.m) * o.d - 1
    assert abs(o.phi_bar * N / (o.n * o.m) - 0.5) < 0.02
    pr = gen_tiny("negbin", n=600, m=400, d=2, R=1, S=1, seed=78)
    t = pr.true
    o = G.OracleGMF(G.Config(family="negbin", link="log", nb_alpha=1.0, R=1, S=1, rate0=1.0,
                             decay=0.0, estimate_alpha=True), pr.Y, pr.X, pr.Z, t["B"],
                    t["A"] + 1.0, t["U"], t["V"])
    o.step()
    assert abs(o.alpha_bar - 5.0) < 0.5


def test_estimates_are_smoothed_with_the_step_size():
    """phi_bar <- (1 - rho_t) phi_bar + rho_t phi^: a second step's value is
    the rho_2-weighted mix of the first value and the new block estimate."""
    pr = gen_tiny("gamma", n=12, m=10, R=2, S=1)
    kw = dict(estimate_phi=True, rate0=0.3, decay=0.5, tau=0.75)
    o = _oracle(pr, R=2, S=1, **kw)
    o.step()
    p1 = o.phi_bar
    r2, _ = o.block_of_step(2)
    probe = copy.deepcopy(o)
    probe.phi_bar = 123.0                 # the block estimate does not depend on phi_bar
    probe.cfg = copy.deepcopy(o.cfg)
    probe.cfg.rate0, probe.cfg.decay = 1.0, 0.0
    probe.step_block(2, r2, 0)
    o.step()
    rho2 = G.learning_rate(o.cfg, 2)
    np.testing.assert_allclose(o.phi_bar, (1 - rho2) * p1 + rho2 * probe.phi_bar, rtol=1e-12)


def test_heldout_metrics_special_cases():
    rng = np.random.default_rng(3)
    y = rng.poisson(2.0, 500).astype(float)
    ybar = 1.7
    e, dp, df = G.heldout_metrics("negbin", y, np.full_like(y, ybar), ybar)
    assert np.isclose(e, 1.0) and np.isclose(dp, 1.0) and np.isclose(df, 1.0)
    e, dp, df = G.heldout_metrics("negbin", y, y, ybar)
    assert e == 0.0 and abs(dp) < 1e-15 and abs(df) < 1e-15
    e, dp, _ = G.heldout_metrics("poisson", y, 0.5 * y + 0.5 * ybar, ybar)
    assert 0 < e < 1 and 0 < dp < 1
