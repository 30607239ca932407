"""The paper's initialization (Section 4.1, least-squares form) on the device
(gmf_initialize) against the FP64 oracle (oracle/init_oracle.py) from the same
test matrix: the column and row effects element by element, the scores and
loadings through what is unique (U V', and U up to the sign of each column),
plus the exact reconstruction of a Gaussian matrix that is exactly low rank
plus intercepts."""
import numpy as np
import pytest

from oracle import gmf_oracle as G
from oracle import init_oracle as I
from synth import gen_nb, gen_tiny

from tests.gpu_helpers import gpu_for, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_20509_amd import gmf  # noqa: F401  raises if libgmf.so is missing


def _compare(g, pr, cfg, Om, power_iters, residual, tol_bg=2e-5, tol_uv=2e-4):
    g.initialize(Om, power_iters=power_iters, residual=residual)
    B, A, U, V = g.params()
    Bo, Ao, Uo, Vo = I.initialize(cfg, pr.Y, pr.X, pr.Z, pr.d, Om, power_iters=power_iters,
                                  residual=residual, W=pr.W)
    eB, eA = rel_err(B, Bo), rel_err(A, Ao)
    UV, UVo = U.astype(np.float64) @ V.astype(np.float64).T, Uo @ Vo.T
    eUV = rel_err(UV, UVo)
    sgn = np.sign(np.sum(U * Uo, axis=0))
    eU = rel_err(U * sgn, Uo)
    print(f"init errors: B {eB:.2e} Gamma {eA:.2e} UV' {eUV:.2e} U {eU:.2e}")
    assert eB <= tol_bg and eA <= tol_bg
    assert eUV <= tol_uv and eU <= tol_uv
    assert np.allclose(np.linalg.norm(U, axis=0), np.linalg.norm(V, axis=0), rtol=1e-5)
    return B, A, U, V


@pytest.mark.parametrize("family,residual", [("negbin", "pearson"), ("poisson", "pearson"),
                                             ("negbin", "deviance")])
def test_initialization_matches_oracle(family, residual):
    print(f"[case] gmf_initialize {family} {residual}", flush=True)
    # ragged: row blocks of 259 rows and column blocks of 166/167 columns
    pr = gen_nb(n=777, m=333, d=4, R=3, S=2, seed=1971, family=family)
    cfg = G.Config(family=pr.family, link=pr.link, nb_alpha=pr.nb_alpha)
    Om = np.random.default_rng(7).normal(size=(pr.m, pr.d + 6)).astype(np.float32)
    g = gpu_for(pr)
    _compare(g, pr, cfg, Om.astype(np.float64), 2, residual)
    # a fit continues from the initialization: its first step matches the
    # oracle's step from the same (device) starting values
    B, A, U, V = g.params()
    o = G.OracleGMF(G.Config(family=pr.family, link=pr.link, nb_alpha=pr.nb_alpha, R=pr.R,
                             S=pr.S, seed=pr.sched_seed), pr.Y, pr.X, pr.Z, B, A, U, V)
    o.step()
    g.step(1)
    B1, A1, U1, V1 = g.params()
    for x, ref in ((B1, o.B), (A1, o.A), (U1, o.U), (V1, o.V)):
        assert rel_err(x, ref) <= 1e-5
    g.close()


def test_initialization_large_ragged_shape():
    """Several row chunks and column tiles per block: 5000 x 1250, 2 x 3 blocks,
    k = 16, weights."""
    print("[case] gmf_initialize 5000x1250 with weights", flush=True)
    pr = gen_tiny("negbin", n=5000, m=1250, d=6, p=2, q=1, R=2, S=3, seed=1972, weights=True)
    cfg = G.Config(family=pr.family, link=pr.link, nb_alpha=pr.nb_alpha)
    Om = np.random.default_rng(8).normal(size=(pr.m, 16)).astype(np.float32)
    g = gpu_for(pr)
    _compare(g, pr, cfg, Om.astype(np.float64), 1, "pearson")
    g.close()


def test_gaussian_exact_low_rank_is_reproduced():
    print("[case] gmf_initialize Gaussian exact low rank", flush=True)
    rng = np.random.default_rng(9)
    n, m, d = 500, 230, 3
    X, Z = np.ones((n, 1)), np.ones((m, 1))
    Y = (X @ rng.normal(size=(m, 1)).T + rng.normal(size=(n, 1)) @ Z.T
         + rng.normal(size=(n, d)) @ rng.normal(size=(m, d)).T).astype(np.float32)
    from paper_2412_20509_amd.gmf import GMF, FitConfig
    g = GMF(FitConfig(family="gaussian", link="identity", d=d, R=2, S=2), Y, X, Z,
            np.zeros((m, 1)), np.zeros((n, 1)), np.zeros((n, d)), np.zeros((m, d)))
    g.initialize(rng.normal(size=(m, d + 4)), power_iters=1)
    B, A, U, V = g.params()
    eta = X @ B.T + A @ Z.T + U.astype(np.float64) @ V.astype(np.float64).T
    err = rel_err(eta, Y)
    print(f"Gaussian low-rank reconstruction error {err:.2e}")
    assert err <= 2e-5
    g.close()


def test_initialization_argument_errors():
    from paper_2412_20509_amd.gmf import GMFError
    pr = gen_nb(n=300, m=200, d=3, R=2, S=2, seed=1973)
    g = gpu_for(pr)
    with pytest.raises(GMFError):
        g.initialize(np.zeros((pr.m, pr.d - 1)))       # k < d
    g.step(1)
    with pytest.raises(GMFError):
        g.initialize(np.random.default_rng(1).normal(size=(pr.m, pr.d + 2)))   # after a step
    g.close()
