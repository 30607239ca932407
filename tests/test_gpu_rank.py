"""Rank selection (Section 4.2) on the device against the oracle: the
singular values of the initialization's residual matrix, the eigenvalue-gap
rank of a planted low-rank count matrix, and the out-of-sample criterion run
through the batched engine (every candidate rank and fold in one batch of
fits with held-out entries missing)."""
import numpy as np
import pytest

from oracle import gmf_oracle as G
from oracle import init_oracle as I
from oracle import rank_oracle as K
from synth import gen_nb

from tests.gpu_helpers import gpu_for, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_20509_amd import gmf  # noqa: F401  raises if libgmf.so is missing


def test_init_spectrum_and_eigengap_rank():
    """A Gaussian matrix with two covariates, a row intercept and a planted
    rank-4 signal under unit noise: the residual matrix's leading singular
    values from the device's range finder match the oracle's exact SVD of the
    same residual matrix, and the eigenvalue gap finds 4.  (On low-count NB
    data the least-squares residuals of the log-transformed counts carry extra
    components, so the gap is not sharp there; the spectrum parity is checked
    on such data too.)"""
    print("[case] residual spectrum and eigen-gap rank", flush=True)
    from paper_2412_20509_amd.gmf import GMF, FitConfig, rank_eigengap
    rng = np.random.default_rng(2301)
    n, m, d = 1500, 700, 4
    X = np.column_stack([np.ones(n), rng.normal(size=n)]).astype(np.float32).astype(np.float64)
    Z = np.ones((m, 1))
    Y = (X @ rng.normal(size=(m, 2)).T + rng.normal(size=(n, 1)) @ Z.T
         + 0.3 * rng.normal(size=(n, d)) @ rng.normal(size=(m, d)).T + rng.normal(size=(n, m)))
    Y = Y.astype(np.float32).astype(np.float64)
    k = 24
    Om = np.random.default_rng(31).normal(size=(m, k)).astype(np.float32)
    g = GMF(FitConfig(family="gaussian", link="identity", d=d, R=3, S=2), Y, X, Z,
            np.zeros((m, 2)), np.zeros((n, 1)), np.zeros((n, d)), np.zeros((m, d)))
    g.initialize(Om, power_iters=4)
    sv = np.asarray(g.init_spectrum(k))
    B = np.linalg.lstsq(X, Y, rcond=None)[0].T
    A = np.linalg.lstsq(Z, (Y - X @ B.T).T, rcond=None)[0].T
    ref = np.linalg.svd(Y - X @ B.T - A @ Z.T, compute_uv=False)
    print("leading singular values:", sv[:6], ref[:6])
    assert rel_err(sv[:4], ref[:4]) <= 1e-5
    # the whole estimated spectrum equals the oracle's range finder from the same Omega
    E = Y - X @ B.T - A @ Z.T
    assert rel_err(sv, I.randomized_singular_values(E, Om.astype(np.float64), 4)) <= 1e-5
    lam = sv ** 2
    assert rank_eigengap(lam, 12) == K.eigengap_rank(lam, 12) == 4
    g.close()
    # NB counts: the spectrum still matches the oracle's residual matrix
    pr = gen_nb(n=1500, m=700, d=4, R=3, S=2, seed=2301)
    g = gpu_for(pr)
    g.initialize(Om, power_iters=6)
    sv = np.asarray(g.init_spectrum(k))
    L = I.link_transform("log", pr.Y)
    B = np.linalg.lstsq(pr.X, L, rcond=None)[0].T
    A = np.linalg.lstsq(pr.Z, (L - pr.X @ B.T).T, rcond=None)[0].T
    mu0 = G.inverse_link("log", pr.X @ B.T + A @ pr.Z.T)
    ref = I.randomized_singular_values(I.residuals("pearson", "negbin", pr.Y, mu0, pr.nb_alpha),
                                       Om.astype(np.float64), 6)
    assert rel_err(sv, ref) <= 2e-4
    g.close()


def test_cv_rank_selection_on_the_batched_engine():
    """A Gaussian matrix of rank 3 plus noise; two folds of 20 % held-out
    entries; ranks 1-6 and both folds run as one batch of 12 fits; the held-out
    deviance is smallest at rank 3, and each fit's held-out deviance matches
    the oracle's fit of the same fold and start."""
    print("[case] cross-validated rank selection, 12 batched fits", flush=True)
    from paper_2412_20509_amd.gmf import FitConfig, cv_rank_table
    rng = np.random.default_rng(5)
    n, m, d = 400, 300, 3
    X, Z = np.ones((n, 1)), np.ones((m, 1))
    Y = rng.normal(size=(n, d)) @ rng.normal(size=(m, d)).T + 0.5 * rng.normal(size=(n, m)) + 1.0
    Y = Y.astype(np.float32).astype(np.float64)
    folds = [rng.random(size=Y.shape) < 0.2 for _ in range(2)]
    starts = {}
    for dd in range(1, 7):
        r = np.random.default_rng(100 + dd)
        starts[dd] = (r.normal(0, 0.1, size=(n, dd)).astype(np.float32).astype(np.float64),
                      r.normal(0, 0.1, size=(m, dd)).astype(np.float32).astype(np.float64))
    fc = FitConfig(family="gaussian", link="identity", R=2, S=2, seed=9, lam=(0, 0, 0.1, 0.1),
                   rate0=0.3, decay=0.05)
    B0, A0 = np.ones((m, 1)), np.zeros((n, 1))
    ranks, table, best = cv_rank_table(fc, Y, X, Z, B0, A0, starts, folds, 40)
    print("held-out deviance by rank:", dict(zip(ranks, table.mean(1).round(4))))
    assert best == 3
    cfg = G.Config(family="gaussian", link="identity", R=2, S=2, seed=9, lam=(0, 0, 0.1, 0.1),
                   rate0=0.3, decay=0.05)
    for dd in (2, 3, 5):
        U0, V0 = starts[dd]
        ref = K.cv_deviance(cfg, Y, X, Z, B0, A0, U0, V0, folds[0], 40)[2]
        assert rel_err([table[ranks.index(dd), 0]], [ref]) <= 2e-3, (dd, table[ranks.index(dd), 0], ref)
