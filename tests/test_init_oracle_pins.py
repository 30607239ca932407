"""Pins of the initialization oracle (Section 4.1, least-squares form) against
what the mathematics fixes: least-squares residuals orthogonal to the
regressors, the randomized range finder equal to the exact truncated SVD when
the residual matrix has rank at most k, Pearson residuals against the moments
of scipy.stats, deviance residuals squaring to the unit deviance, and an exact
reconstruction of a Gaussian matrix that is exactly low rank plus intercepts."""
import numpy as np
import pytest
from scipy import stats

from oracle import gmf_oracle as G
from oracle import init_oracle as I


def _rng(seed):
    return np.random.default_rng(seed)


def test_link_transform():
    y = np.array([[0, 1, 7]], dtype=np.float64)
    assert np.allclose(I.link_transform("log", y), np.log(y + 0.5))
    assert np.allclose(I.link_transform("log", y, offset=1.0), np.log1p(y))
    assert np.allclose(I.link_transform("identity", y), y)


def test_pearson_residuals_match_scipy_moments():
    mu = np.array([0.05, 0.3, 2.0, 17.0])
    y = np.array([0.0, 2.0, 1.0, 30.0])
    a = 5.0
    m_p, v_p = stats.poisson.stats(mu, moments="mv")
    m_nb, v_nb = stats.nbinom.stats(a, a / (a + mu), moments="mv")
    assert np.allclose(m_p, mu) and np.allclose(m_nb, mu)
    assert np.allclose(I.residuals("pearson", "poisson", y, mu), (y - mu) / np.sqrt(v_p), rtol=1e-13)
    assert np.allclose(I.residuals("pearson", "negbin", y, mu, a), (y - mu) / np.sqrt(v_nb),
                       rtol=1e-13)
    w = np.array([0.5, 1.0, 2.0, 3.0])
    assert np.allclose(I.residuals("pearson", "negbin", y, mu, a, W=w),
                       (y - mu) / np.sqrt(v_nb / w), rtol=1e-13)
    assert np.allclose(I.residuals("pearson", "gaussian", y, mu), y - mu)


def test_deviance_residuals_square_to_unit_deviance():
    mu = np.array([0.05, 0.3, 2.0, 17.0, 4.0])
    y = np.array([0.0, 2.0, 1.0, 30.0, 4.0])
    for fam in ("poisson", "negbin", "gaussian"):
        r = I.residuals("deviance", fam, y, mu, 5.0)
        assert np.allclose(r ** 2, G.unit_deviance(fam, y, mu, 5.0), rtol=1e-12, atol=1e-300)
        assert np.all(np.sign(r) == np.sign(y - mu))


def test_range_finder_is_exact_svd_for_low_rank():
    """A residual matrix of rank r <= k: the range of E Omega is the range of E,
    so the randomized vectors are the exact leading singular vectors (up to
    sign), with any number of power iterations."""
    rng = _rng(3)
    n, m, r, d, k = 300, 120, 6, 4, 9
    sv = np.array([50.0, 30.0, 20.0, 12.0, 5.0, 2.0])
    P = np.linalg.qr(rng.normal(size=(n, r)))[0]
    Q = np.linalg.qr(rng.normal(size=(m, r)))[0]
    E = (P * sv) @ Q.T
    Om = rng.normal(size=(m, k))
    for it in (0, 1, 3):
        U = I.randomized_left_vectors(E, Om, it, d)
        Ue = np.linalg.svd(E, full_matrices=False)[0][:, :d]
        assert np.allclose(np.abs(U.T @ Ue), np.eye(d), atol=1e-10)


def test_range_finder_with_a_planted_gap_approaches_eckart_young():
    """Full-rank noise below a planted rank-d signal: with power iterations the
    captured energy ||U U'E||_F^2 approaches the Eckart-Young optimum (the sum
    of the d largest squared singular values) and the error shrinks with q."""
    rng = _rng(4)
    n, m, d, k = 400, 200, 3, 8
    P = np.linalg.qr(rng.normal(size=(n, d)))[0]
    Q = np.linalg.qr(rng.normal(size=(m, d)))[0]
    E = (P * np.array([40.0, 25.0, 15.0])) @ Q.T + 0.05 * rng.normal(size=(n, m))
    s = np.linalg.svd(E, compute_uv=False)
    best = np.sum(s[:d] ** 2)
    Om = rng.normal(size=(m, k))
    gaps = []
    for it in (0, 1, 2):
        U = I.randomized_left_vectors(E, Om, it, d)
        gaps.append(best - np.sum((U.T @ E) ** 2))
    assert all(g >= -1e-9 * best for g in gaps)
    assert gaps[2] <= 1e-10 * best
    assert gaps[2] <= gaps[0]


def _problem(seed, family="poisson", n=180, m=90, d=3):
    rng = _rng(seed)
    X = np.column_stack([np.ones(n), rng.integers(0, 2, n), rng.normal(size=n)])
    Z = np.ones((m, 1))
    eta = (X @ rng.normal(0, 0.4, size=(m, 3)).T + rng.normal(0, 0.3, size=(n, 1)) @ Z.T
           + rng.normal(0, 0.5, size=(n, d)) @ rng.normal(0, 0.5, size=(m, d)).T)
    Y = rng.poisson(np.exp(eta)).astype(np.float64)
    return Y, X, Z, rng.normal(size=(m, d + 5))


@pytest.mark.parametrize("family", ["poisson", "negbin"])
@pytest.mark.parametrize("residual", ["pearson", "deviance"])
def test_least_squares_steps_are_orthogonal_projections(family, residual):
    Y, X, Z, Om = _problem(5)
    cfg = G.Config(family=family, link="log")
    d = 3
    # enough power iterations that the range finder converges on this noisy
    # residual matrix (no planted gap), so that U can be checked against the SVD
    B, A, U, V = I.initialize(cfg, Y, X, Z, d, Om, power_iters=12, residual=residual)
    L = I.link_transform("log", Y)
    R1 = L - X @ B.T
    assert np.max(np.abs(X.T @ R1)) <= 1e-10 * np.max(np.abs(X.T @ L))
    R2 = R1 - A @ Z.T
    assert np.max(np.abs(R2 @ Z)) <= 1e-10 * np.max(np.abs(R1 @ Z) + 1)
    # the loadings solve the normal equations of the link-scale residual on U
    assert np.max(np.abs(U.T @ (R2 - U @ V.T))) <= 1e-9 * np.max(np.abs(U.T @ R2))
    # equal norms within each pair
    assert np.allclose(np.linalg.norm(U, axis=0), np.linalg.norm(V, axis=0), rtol=1e-12)
    # U spans the leading left singular subspace of the residual matrix
    mu0 = G.inverse_link("log", X @ B.T + A @ Z.T)
    E = I.residuals(residual, family, Y, mu0, cfg.nb_alpha)
    Ue = np.linalg.svd(E, full_matrices=False)[0][:, :d]
    Un = U / np.linalg.norm(U, axis=0)
    cos = np.linalg.svd(Un.T @ Ue, compute_uv=False)
    assert cos.min() > 1 - 1e-6


def test_gaussian_exact_low_rank_is_reproduced():
    """Y = 1 beta0' + gamma0 1' + U V' exactly (identity link): the column and
    row least squares remove the intercepts, the double-centred residual has
    rank d, so the initialization reproduces Y exactly."""
    rng = _rng(6)
    n, m, d = 150, 70, 3
    X, Z = np.ones((n, 1)), np.ones((m, 1))
    Y = (X @ rng.normal(size=(m, 1)).T + rng.normal(size=(n, 1)) @ Z.T
         + rng.normal(size=(n, d)) @ rng.normal(size=(m, d)).T)
    cfg = G.Config(family="gaussian", link="identity")
    B, A, U, V = I.initialize(cfg, Y, X, Z, d, rng.normal(size=(m, d + 4)), power_iters=1)
    eta = X @ B.T + A @ Z.T + U @ V.T
    assert np.max(np.abs(eta - Y)) <= 1e-10 * np.max(np.abs(Y))
    # with one factor too few the reconstruction is the best rank-(d-1) one
    B, A, U, V = I.initialize(cfg, Y, X, Z, d - 1, rng.normal(size=(m, d + 4)), power_iters=2)
    Rc = Y - Y.mean(0) - Y.mean(1, keepdims=True) + Y.mean()
    s = np.linalg.svd(Rc, compute_uv=False)
    err = np.sum((Y - X @ B.T - A @ Z.T - U @ V.T) ** 2)
    assert abs(err - s[d - 1] ** 2) <= 1e-8 * s[0] ** 2


def test_logit_transform_maps_binary_values():
    y = np.array([0.0, 1.0])
    np.testing.assert_allclose(I.link_transform("logit", y), [-np.log(3.0), np.log(3.0)],
                               rtol=1e-14)
