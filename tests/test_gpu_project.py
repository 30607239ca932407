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
