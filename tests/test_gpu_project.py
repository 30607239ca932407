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


def _first_within(trace, target, rel):
    for e, v in enumerate(trace):
        if abs(v - target) <= rel * target:
            return e
    return None


def test_trained_encoder_gains_epochs_over_cold_start():
    """What the learned part gains (the warm start of new rows).  The column
    side is the oracle's 30-epoch fit of a 3000 x 700 NB problem, handed to the
    library with gmf_set_params and frozen at its Algorithm 2 form; the encoder
    is trained on the library's converged projections of the fitted rows; the
    1500 new rows are fresh draws with the same true column side.  The target
    D* is the deviance of the new rows at the oracle's own projection run to
    convergence (200 epochs from the cold start).  The warm start from the
    trained encoder's bfloat16 predictions must reach 1e-4 of D* in at most
    0.75 times the cold start's epochs, with few fallback rows; an untrained
    encoder of the same shape (random starting weights) falls back to the cold
    start on a large share of the rows and does not reach that gain."""
    print("[case] trained encoder vs cold start vs untrained encoder", flush=True)
    from paper_2412_20509_amd.gmf import Encoder
    from synth import gen_nb_rows, mlp_init
    pr = gen_nb(n=3000, m=700, d=6, R=3, S=4, seed=1047)
    o = oracle_for(pr)
    o.steps(30 * pr.R * pr.S)
    g = gpu_for(pr)
    g.set_params(o.B, o.A, o.U, o.V)
    cfg = _cfg(pr)
    Bf, _, _, Vf = G.postprocess_A_B1(pr.X, pr.Z, o.B, o.A, o.U, o.V)
    # encoder targets: the fitted rows' own projections run to convergence
    _, Ut, _, _, _ = g.project_warm(pr.Y, pr.X, None, 80, frozen=1)
    enc = Encoder(pr.m, pr.d, mlp_init(pr.m, 64, pr.d, seed=9), hidden=64, batch=128, lr=2e-3)
    tr = enc.train(pr.Y, Ut, 40)
    assert tr[-1] < 0.2 * tr[0], tr
    Ynew, Xnew, _, _ = gen_nb_rows(pr, 1500, seed=5047)
    Ynew = np.asarray(Ynew)
    Xnew = np.asarray(Xnew, np.float64)
    # D*: the oracle's projection of the new rows from the cold start
    cols = G.partition(G.permutation(cfg.seed, G.STREAM_COLS, pr.m), pr.S)
    A0 = G.row_intercept_start(cfg, Ynew, Xnew, Bf, pr.q)
    Ao, Uo = G.project_rows(cfg, Ynew, Xnew, pr.Z, Bf, Vf, A0, np.zeros((len(Ynew), pr.d)),
                            200, cols)
    dstar = G.row_deviance(cfg, Ynew, Xnew, pr.Z, Bf, Ao, Uo, Vf).sum()
    epochs = 60
    _, _, trc, _, fbc = g.project_warm(Ynew, Xnew, None, epochs, frozen=1, trace=True)
    cand = enc.forward(Ynew, bf16=True)
    _, _, trw, _, fbw = g.project_warm(Ynew, Xnew, cand, epochs, frozen=1, trace=True)
    ec, ew = _first_within(trc, dstar, 1e-4), _first_within(trw, dstar, 1e-4)
    print(f"epochs to 1e-4 of D*: cold {ec}, warm {ew}; fallback rows {fbw} of {len(Ynew)}; "
          f"start deviances cold {trc[0]:.1f} warm {trw[0]:.1f} D* {dstar:.1f}")
    assert fbc == 0
    assert ec is not None and ew is not None
    assert ew <= 0.75 * ec
    assert fbw < 0.1 * len(Ynew)
    # control: the same encoder shape with its untrained random weights gains
    # nothing comparable: about half of its rows fall back to the cold start
    # and it needs more than 0.75 times the cold start's epochs
    enc0 = Encoder(pr.m, pr.d, mlp_init(pr.m, 64, pr.d, seed=9), hidden=64, batch=128, lr=2e-3)
    cand0 = enc0.forward(Ynew, bf16=True)
    _, _, tr0, _, fb0 = g.project_warm(Ynew, Xnew, cand0, epochs, frozen=1, trace=True)
    e0 = _first_within(tr0, dstar, 1e-4)
    print(f"untrained encoder: {fb0} fallback rows of {len(Ynew)}, {e0} epochs to 1e-4 of D*")
    assert fb0 > 0.3 * len(Ynew)
    assert e0 is None or e0 > 0.75 * ec
    enc0.close()
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
