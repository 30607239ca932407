"""The allocation-free projection (gmf_project_noalloc, resident scratch)
against gmf_project (caller workspace) on the same context: the same kernels on
the same inputs, so the results must be bit-identical; two calls in a row, the
second with fewer rows (the scratch keeps the first call's contents), plus a
call beyond the scratch limit, which must be refused."""
import numpy as np
import pytest

from synth import gen_nb

from tests.gpu_helpers import gpu_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_20509_amd import gmf  # noqa: F401  raises if libgmf.so is missing


@pytest.mark.parametrize("frozen", [0, 1])
def test_noalloc_projection_equals_workspace_projection(frozen):
    print(f"[case] gmf_project_noalloc vs gmf_project, frozen={frozen}", flush=True)
    pr = gen_nb(n=2400, m=700, d=6, R=3, S=4, seed=1061)
    new = gen_nb(n=1800, m=700, d=6, R=3, S=4, seed=1562)
    g = gpu_for(pr)
    g.step(2 * pr.R * pr.S)
    rng = np.random.default_rng(5)
    A0 = rng.normal(0, 0.1, size=(new.n, pr.q))
    U0 = rng.normal(0, 0.1, size=(new.n, pr.d))
    for rows in (np.arange(new.n), np.arange(150, 1333)):       # second call smaller
        Y, X = new.Y[rows], new.X[rows]
        Aw, Uw, trw = g.project(Y, X, A0[rows], U0[rows], 3, frozen=frozen, trace=True)
        An, Un, trn = g.project_noalloc(Y, X, A0[rows], U0[rows], 3, frozen=frozen, trace=True)
        assert np.array_equal(An.cpu().numpy(), Aw.cpu().numpy())
        assert np.array_equal(Un.cpu().numpy(), Uw.cpu().numpy())
        assert trn == trw
    g.close()


def test_noalloc_projection_refuses_more_than_its_scratch():
    from paper_2412_20509_amd.gmf import GMFError
    print("[case] gmf_project_noalloc size limit", flush=True)
    pr = gen_nb(n=600, m=2000, d=4, R=2, S=2, seed=1063)
    g = gpu_for(pr)
    n_new = 9000                        # 9000 x 2000 floats of counts alone: 72 MB
    Y = np.zeros((n_new, pr.m), np.int32)
    X = np.ones((n_new, pr.p))
    with pytest.raises(GMFError):
        g.project_noalloc(Y, X, np.zeros((n_new, pr.q)), np.zeros((n_new, pr.d)), 1)
    g.close()
