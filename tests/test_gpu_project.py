"""Projection of new rows with the column side frozen (gmf_project) against the
oracle's row-side iteration, plus its structural properties."""
import numpy as np
import pytest

from oracle import gmf_oracle as G
from synth import gen_nb

from tests.gpu_helpers import gpu_for, oracle_for, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _fit_and_new_rows(seed=1041):
    pr = gen_nb(n=3000, m=700, d=6, R=3, S=4, seed=seed)
    new = gen_nb(n=1500, m=700, d=6, R=3, S=4, seed=seed + 500)   # new rows, own draw
    g = gpu_for(pr)
    g.step(3 * pr.R * pr.S)
    return pr, new, g


def _oracle_project(pr, new, B, V, epochs):
    cfg = G.Config(family=pr.family, link=pr.link, nb_alpha=pr.nb_alpha, R=pr.R, S=pr.S,
                   seed=pr.sched_seed)
    cols = G.partition(G.permutation(cfg.seed, G.STREAM_COLS, pr.m), pr.S)
    A0 = np.zeros((new.n, pr.q))
    U0 = np.zeros((new.n, pr.d))
    return G.project_rows(cfg, new.Y, new.X, pr.Z, B, V, A0, U0, epochs, cols)


@pytest.mark.parametrize("frozen", [0, 1])
def test_projection_matches_oracle(frozen):
    print(f"[case] projection frozen={frozen}", flush=True)
    pr, new, g = _fit_and_new_rows()
    B, A, U, V = g.params(0)
    if frozen:
        B, _, _, V = G.postprocess_A_B1(pr.X, pr.Z, B, A, U, V)
    A0 = np.zeros((new.n, pr.q))
    U0 = np.zeros((new.n, pr.d))
    Ag, Ug, tr = g.project(new.Y, new.X, A0, U0, 4, frozen=frozen, trace=True)
    Ao, Uo = _oracle_project(pr, new, B, V, 4)
    assert rel_err(Ag.cpu().numpy(), Ao) <= 2e-4
    assert rel_err(Ug.cpu().numpy(), Uo) <= 2e-4
    # the deviance of the new rows never rises across epochs here
    assert all(b <= a * (1 + 1e-6) for a, b in zip(tr, tr[1:])), tr
    # and it equals the oracle's deviance of the projected rows
    dev_o = G.row_deviance(G.Config(family="negbin", nb_alpha=pr.nb_alpha), new.Y, new.X, pr.Z,
                           B, Ao, Uo, V).sum()
    assert abs(tr[-1] - dev_o) <= 1e-4 * dev_o
    g.close()


def test_projection_rows_are_independent():
    print("[case] projection row independence", flush=True)
    pr, new, g = _fit_and_new_rows(1042)
    A0 = np.zeros((new.n, pr.q))
    U0 = np.zeros((new.n, pr.d))
    Ag, Ug, _ = g.project(new.Y, new.X, A0, U0, 3)
    sub = np.arange(100, 700)
    As, Us, _ = g.project(new.Y[sub], new.X[sub], A0[sub], U0[sub], 3)
    assert np.array_equal(As.cpu().numpy(), Ag.cpu().numpy()[sub])
    assert np.array_equal(Us.cpu().numpy(), Ug.cpu().numpy()[sub])
    g.close()


# ------------------------------------------------ warm-start starting values --

def _cfg(pr):
    return G.Config(family=pr.family, link=pr.link, nb_alpha=pr.nb_alpha, R=pr.R, S=pr.S,
                    seed=pr.sched_seed)


def _candidates(pr, new, B, V):
    """Good candidate scores (the oracle's 3-epoch projection) on two rows in
    three, poor ones (N(0, 1.5^2)) on the rest."""
    _, Uo = _oracle_project(pr, new, B, V, 3)
    cand = Uo.copy()
    rng = np.random.default_rng(77)
    cand[::3] = rng.normal(0.0, 1.5, size=cand[::3].shape)
    return cand.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("frozen", [0, 1])
def test_warm_start_values_match_oracle(frozen):
    print(f"[case] warm start values frozen={frozen}", flush=True)
    pr, new, g = _fit_and_new_rows(1043)
    B, A, U, V = g.params(0)
    if frozen:
        B, _, _, V = G.postprocess_A_B1(pr.X, pr.Z, B, A, U, V)
    cfg = _cfg(pr)
    cand = _candidates(pr, new, B, V)
    Ag, Ug, tr, ms, fb = g.project_warm(new.Y, new.X, cand, 0, frozen=frozen, trace=True)
    Ag, Ug = Ag.cpu().numpy().astype(np.float64), Ug.cpu().numpy().astype(np.float64)
    A0o = G.row_intercept_start(cfg, new.Y, new.X, B, pr.q)
    assert rel_err(Ag, A0o) <= 1e-5
    U0o, warm, dc, d0 = G.warm_start_rows(cfg, new.Y, new.X, pr.Z, B, V, A0o, cand)
    clear = np.abs(dc - d0) > 1e-4 * d0          # rows whose choice rounding cannot flip
    assert clear.mean() > 0.9
    gpu_warm = np.any(Ug != 0.0, axis=1)
    assert np.array_equal(gpu_warm[clear], warm[clear])
    assert np.array_equal(Ug[gpu_warm], cand[gpu_warm])         # chosen rows: exactly the candidate
    assert fb == int((~gpu_warm).sum())
    assert 0 < fb < new.n
    # the deviance before the first step is that of the chosen starting values
    dev0 = G.row_deviance(cfg, new.Y, new.X, pr.Z, B, A0o, U0o, V)
    assert abs(tr[0] - dev0.sum()) <= 1e-5 * dev0.sum()
    assert len(ms) == 1 and ms[0] > 0
    g.close()


def test_warm_projection_trajectory_matches_oracle():
    print("[case] warm projection 3 epochs vs oracle", flush=True)
    pr, new, g = _fit_and_new_rows(1044)
    B, A, U, V = g.params(0)
    B, _, _, V = G.postprocess_A_B1(pr.X, pr.Z, B, A, U, V)
    cfg = _cfg(pr)
    cand = _candidates(pr, new, B, V)
    A0o = G.row_intercept_start(cfg, new.Y, new.X, B, pr.q)
    U0o, warm, dc, d0 = G.warm_start_rows(cfg, new.Y, new.X, pr.Z, B, V, A0o, cand)
    Ag, Ug, tr, ms, fb = g.project_warm(new.Y, new.X, cand, 3, frozen=1, trace=True)
    cols = G.partition(G.permutation(cfg.seed, G.STREAM_COLS, pr.m), pr.S)
    Ao, Uo = G.project_rows(cfg, new.Y, new.X, pr.Z, B, V, A0o, U0o, 3, cols)
    clear = np.abs(dc - d0) > 1e-4 * d0
    assert rel_err(Ag.cpu().numpy()[clear], Ao[clear]) <= 2e-4
    assert rel_err(Ug.cpu().numpy()[clear], Uo[clear]) <= 2e-4
    assert len(tr) == 4 and all(b <= a * (1 + 1e-6) for a, b in zip(tr, tr[1:])), tr
    assert all(b > a for a, b in zip(ms, ms[1:]))
    g.close()


def test_cold_start_is_intercept_and_zero_scores():
    print("[case] cold start values and consistency with gmf_project", flush=True)
    pr, new, g = _fit_and_new_rows(1045)
    B, A, U, V = g.params(0)
    cfg = _cfg(pr)
    A0g, U0g, _, _, fb = g.project_warm(new.Y, new.X, None, 0, frozen=0)
    assert fb == 0
    assert np.all(U0g.cpu().numpy() == 0.0)
    assert rel_err(A0g.cpu().numpy(), G.row_intercept_start(cfg, new.Y, new.X, B, pr.q)) <= 1e-5
    # the same epochs from the same starting values as gmf_project: identical
    A2, U2, _, _, _ = g.project_warm(new.Y, new.X, None, 2, frozen=0)
    A3, U3, _ = g.project(new.Y, new.X, A0g, U0g, 2, frozen=0)
    assert np.array_equal(A2.cpu().numpy(), A3.cpu().numpy())
    assert np.array_equal(U2.cpu().numpy(), U3.cpu().numpy())
    g.close()


def test_encoder_warm_start_end_to_end():
    """Fit, train the encoder on the fitted (Algorithm 2) scores, warm-start new
    rows from its bfloat16 predictions: by the per-row selection the warm
    start's deviance is never above the cold start's."""
    print("[case] encoder warm start end to end", flush=True)
    from paper_2412_20509_amd.gmf import Encoder
    from synth import mlp_init
    pr, new, g = _fit_and_new_rows(1046)
    _, _, Ufit, _ = g.params(1)
    enc = Encoder(pr.m, pr.d, mlp_init(pr.m, 64, pr.d, seed=9), hidden=64, batch=128, lr=2e-3)
    tr = enc.train(pr.Y, Ufit, 15)
    assert tr[-1] < tr[0]
    cand = enc.forward(new.Y, bf16=True)
    _, _, trw, _, fbw = g.project_warm(new.Y, new.X, cand, 1, frozen=1, trace=True)
    _, _, trc, _, fbc = g.project_warm(new.Y, new.X, None, 1, frozen=1, trace=True)
    assert fbc == 0 and 0 <= fbw < new.n
    assert trw[0] <= trc[0]
    enc.close()
    g.close()


def test_projection_split_bf16_matches_oracle():
    """The projection in split bfloat16 (a context fitted in FP32 with panel
    stride 32, switched with gmf_set_precision): products off by about 2^-17
    relative, gated at 10x the FP32 gate (2e-3); the deviance of the projected
    rows within 1e-4 of the oracle's, as for FP32."""
    print("[case] projection split bf16", flush=True)
    pr = gen_nb(n=3000, m=700, d=6, R=3, S=4, seed=1043)
    new = gen_nb(n=1500, m=700, d=6, R=3, S=4, seed=1543)
    g = gpu_for(pr, panel_stride=32)
    g.step(3 * pr.R * pr.S)
    B, A, U, V = g.params(0)
    B, _, _, V = G.postprocess_A_B1(pr.X, pr.Z, B, A, U, V)
    g.set_precision("bf16x3")
    A0 = np.zeros((new.n, pr.q))
    U0 = np.zeros((new.n, pr.d))
    Ag, Ug, tr = g.project(new.Y, new.X, A0, U0, 4, frozen=1, trace=True)
    Ao, Uo = _oracle_project(pr, new, B, V, 4)
    print("split bf16 projection errors:", rel_err(Ag.cpu().numpy(), Ao), rel_err(Ug.cpu().numpy(), Uo))
    assert rel_err(Ag.cpu().numpy(), Ao) <= 2e-3
    assert rel_err(Ug.cpu().numpy(), Uo) <= 2e-3
    dev_o = G.row_deviance(G.Config(family="negbin", nb_alpha=pr.nb_alpha), new.Y, new.X, pr.Z,
                           B, Ao, Uo, V).sum()
    assert abs(tr[-1] - dev_o) <= 1e-4 * dev_o
    g.close()


@pytest.mark.parametrize("precision", ["bf16x3", "bf16"])
def test_projection_bfloat16_at_stride_16(precision):
    """An FP32 context at panel stride 16 projecting in a bfloat16 precision
    (16x16x16 bfloat16 products).  Split BF16: products off by about 2^-17
    relative, gated like the stride-32 case (2e-3 on the scores, 1e-4 on the
    deviance).  BF16: operands rounded to 8 bits (2^-9 relative), gated like
    the BF16 fit (5e-2 on the scores) and 1e-3 on the deviance of the
    projected rows (the rows converge to a nearby optimum)."""
    print(f"[case] projection {precision} at stride 16", flush=True)
    pr, new, g = _fit_and_new_rows(1044)
    B, A, U, V = g.params(0)
    B, _, _, V = G.postprocess_A_B1(pr.X, pr.Z, B, A, U, V)
    g.set_precision(precision)
    A0 = np.zeros((new.n, pr.q))
    U0 = np.zeros((new.n, pr.d))
    Ag, Ug, tr = g.project(new.Y, new.X, A0, U0, 4, frozen=1, trace=True)
    Ao, Uo = _oracle_project(pr, new, B, V, 4)
    ea, eu = rel_err(Ag.cpu().numpy(), Ao), rel_err(Ug.cpu().numpy(), Uo)
    dev_o = G.row_deviance(G.Config(family="negbin", nb_alpha=pr.nb_alpha), new.Y, new.X, pr.Z,
                           B, Ao, Uo, V).sum()
    ed = abs(tr[-1] - dev_o) / dev_o
    print(f"{precision} stride-16 projection errors: A {ea:.2e} U {eu:.2e} deviance {ed:.2e}")
    tol, tol_d = (2e-3, 1e-4) if precision == "bf16x3" else (5e-2, 1e-3)
    assert ea <= tol and eu <= tol
    assert ed <= tol_d
    g.set_precision("fp32")
    g.close()
