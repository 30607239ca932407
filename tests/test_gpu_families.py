"""The generic epilogue on the device against the oracle: the Gamma, inverse
Gaussian and Bernoulli families (Supplementary Table 1), missing entries
imputed by their mean (Section 3.2.2), per-column NB shapes, the stochastic
dispersion and NB-shape estimators (Appendix B), the held-out metrics of
Section 5.2 and the initialization with missing entries; one step at the
per-step tolerance (1e-5) and one epoch at 2e-4, as for the fast paths."""
import numpy as np
import pytest

from oracle import gmf_oracle as G
from oracle import init_oracle as I
from synth import gen_nb, gen_tiny, holdout

from tests.gpu_helpers import compare_state, gpu_for, oracle_for, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_20509_amd import gmf  # noqa: F401  raises if libgmf.so is missing


def _step_and_epoch(pr, label, o_over=None, g_over=None, Y=None):
    o_over = o_over or {}
    g_over = g_over or {}
    if Y is not None:
        pr.Y = Y
    o = oracle_for(pr, **o_over)
    g = gpu_for(pr, **g_over)
    dev_o = o.step()
    g.step(1)
    compare_state(g, o, 1e-5, f"{label}: one step")
    if not o_over.get("estimate_alpha"):
        assert rel_err([g.block_deviance(1)[0]], [dev_o]) <= 1e-5
    o.steps(pr.R * pr.S - 1)
    g.step(pr.R * pr.S - 1)
    compare_state(g, o, 2e-4, f"{label}: one epoch")
    dg, _ = g.deviance()
    assert rel_err([dg], [o.full_deviance()]) <= 1e-5
    return o, g


@pytest.mark.parametrize("family,weights", [("gamma", True), ("invgauss", False),
                                            ("bernoulli", True)])
def test_new_families_match_oracle(family, weights):
    print(f"[case] generic family {family} weights={weights}", flush=True)
    pr = gen_tiny(family, n=333, m=250, d=4, p=2, q=1, R=3, S=2, seed=2101, weights=weights)
    _, g = _step_and_epoch(pr, family)
    g.close()


@pytest.mark.parametrize("family", ["poisson", "negbin", "gaussian", "gamma"])
def test_missing_entries_match_oracle(family):
    print(f"[case] missing entries {family}", flush=True)
    pr = gen_tiny(family, n=401, m=277, d=3, p=3, q=1, R=3, S=3, seed=2102)
    Yt, _ = holdout(pr.Y, 0.3, seed=2103)
    _, g = _step_and_epoch(pr, f"{family} with 30% missing", g_over=dict(allow_missing=1), Y=Yt)
    # per-row deviances cover the observed entries
    import torch
    rd = g.row_deviance()
    B, A, U, V = g.params()
    cfg = G.Config(family=pr.family, link=pr.link, nb_alpha=pr.nb_alpha)
    ref = G.row_deviance(cfg, Yt, pr.X, pr.Z, B, A, U, V)
    assert rel_err(rd, ref) <= 2e-5
    g.close()


def test_complete_data_generic_path_equals_fast_path():
    """allow_missing on complete data runs the generic epilogue; its steps agree
    with the Poisson fast path to float32 rounding."""
    pr = gen_nb(n=600, m=300, d=4, R=3, S=2, seed=2104, family="poisson")
    a = gpu_for(pr)
    b = gpu_for(pr, allow_missing=1)
    a.step(12)
    b.step(12)
    for x, y in zip(a.params(), b.params()):
        assert rel_err(y, x) <= 1e-6
    a.close()
    b.close()


def test_per_column_nb_shape_matches_oracle():
    print("[case] per-column NB shape", flush=True)
    pr = gen_nb(n=500, m=310, d=4, R=3, S=2, seed=2105)
    alpha = np.linspace(0.5, 20.0, pr.m).astype(np.float32).astype(np.float64)
    o = oracle_for(pr, nb_alpha=alpha)
    g = gpu_for(pr)
    g.set_column_alpha(alpha)
    d0, _ = g.deviance()
    assert rel_err([d0], [o.full_deviance()]) <= 1e-6
    dev_o = o.step()
    g.step(1)
    compare_state(g, o, 1e-5, "per-column alpha, one step")
    assert rel_err([g.block_deviance(1)[0]], [dev_o]) <= 1e-5
    o.steps(pr.R * pr.S - 1)
    g.step(pr.R * pr.S - 1)
    compare_state(g, o, 2e-4, "per-column alpha, one epoch")
    g.close()


@pytest.mark.parametrize("family,flag", [("gamma", "estimate_phi"), ("negbin", "estimate_alpha"),
                                         ("invgauss", "estimate_phi")])
def test_dispersion_estimation_matches_oracle(family, flag):
    print(f"[case] {flag} {family}", flush=True)
    pr = gen_tiny(family, n=380, m=260, d=3, p=2, q=1, R=2, S=2, seed=2106)
    start = dict(phi=1.3) if flag == "estimate_phi" else dict(nb_alpha=2.0)
    o, g = _step_and_epoch(pr, f"{flag} {family}", o_over=dict(start, **{flag: True}),
                           g_over=dict(start, **{flag: 1}))
    phi, alpha = g.dispersion()
    if flag == "estimate_phi":
        assert abs(phi - o.phi_bar) <= 2e-4 * o.phi_bar and phi != 1.3
    else:
        assert abs(alpha - o.alpha_bar) <= 2e-4 * o.alpha_bar and alpha != 2.0
    # resume from a saved state continues bit for bit, estimates included
    state = g.save_state()
    g.step(3)
    ref = g.params()
    h = gpu_for(pr, **dict(start, **{flag: 1}))
    h.load_state(state)
    h.step(3)
    for x, y in zip(ref, h.params()):
        assert np.array_equal(x, y)
    assert h.dispersion() == g.dispersion()
    g.close()
    h.close()


def test_heldout_metrics_match_oracle():
    print("[case] held-out metrics", flush=True)
    pr = gen_nb(n=700, m=420, d=4, R=3, S=3, seed=2107)
    Yt, mask = holdout(pr.Y, 0.3, seed=2108)
    pr.Y = Yt
    g = gpu_for(pr, allow_missing=1)
    g.step(5 * pr.R * pr.S)
    B, A, U, V = g.params()
    eta = pr.X @ B.T + A @ pr.Z.T + U.astype(np.float64) @ V.astype(np.float64).T
    mu = G.inverse_link("log", eta)
    Ytrue = gen_nb(n=700, m=420, d=4, R=3, S=3, seed=2107).Y
    ybar = np.nanmean(Yt)
    ref = G.heldout_metrics("negbin", Ytrue[mask], mu[mask], ybar, pr.nb_alpha)
    Ytest = np.where(mask, Ytrue, -1).astype(np.int32)
    out = g.heldout_metrics(Ytest)
    print("held-out metrics:", out[:3], "oracle:", ref)
    assert rel_err(out[:3], ref) <= 1e-4
    assert out[3] == mask.sum() and abs(out[4] - ybar) <= 1e-9 * ybar
    assert 0 < out[1] < 1
    g.close()


@pytest.mark.parametrize("family", ["negbin", "bernoulli"])
def test_initialization_with_missing_entries_matches_oracle(family):
    print(f"[case] initialization with missing entries, {family}", flush=True)
    pr = gen_tiny(family, n=640, m=300, d=3, p=2, q=1, R=2, S=2, seed=2109)
    Yt, _ = holdout(pr.Y, 0.25, seed=2110)
    pr.Y = Yt
    Om = np.random.default_rng(12).normal(size=(pr.m, pr.d + 5)).astype(np.float32)
    g = gpu_for(pr, allow_missing=1)
    g.initialize(Om, power_iters=2)
    B, A, U, V = g.params()
    cfg = G.Config(family=pr.family, link=pr.link, nb_alpha=pr.nb_alpha)
    Bo, Ao, Uo, Vo = I.initialize(cfg, Yt, pr.X, pr.Z, pr.d, Om.astype(np.float64), power_iters=2)
    print("init errors:", rel_err(B, Bo), rel_err(A, Ao), rel_err(U @ V.T, Uo @ Vo.T))
    assert rel_err(B, Bo) <= 2e-5 and rel_err(A, Ao) <= 2e-5
    assert rel_err(U.astype(np.float64) @ V.astype(np.float64).T, Uo @ Vo.T) <= 2e-4
    g.close()


def test_generic_contexts_refuse_bfloat16_and_projection():
    from paper_2412_20509_amd.gmf import GMFError
    pr = gen_tiny("gamma", n=200, m=120, d=3, p=2, q=1, R=2, S=2, seed=2111)
    g = gpu_for(pr)
    with pytest.raises(GMFError):
        g.set_precision("bf16")
    with pytest.raises(GMFError):
        g.project(pr.Y[:10], pr.X[:10], np.zeros((10, 1)), np.zeros((10, 3)), 1)
    g.close()
    with pytest.raises(GMFError):
        gpu_for(pr, precision="bf16")
