"""The 16-bit copy of the counts (cfg.compact_counts): the step tiles and the
full deviance read it instead of the float32 counts.  The counts are the same
numbers, so every output is the same bits as with the float32 counts: in
every precision, for Poisson and NB, with and without weights, on ragged
blocks.  Counts that do not fit 16 bits, and non-count families, keep the
float32 path."""
import dataclasses

import numpy as np
import pytest

from synth import gen_gaussian_lowrank, gen_nb

from tests.gpu_helpers import gpu_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_20509_amd import gmf  # noqa: F401  raises if libgmf.so is missing


def _run(pr, precision, compact, steps):
    g = gpu_for(pr, precision=precision, compact_counts=compact)
    flag = g.compact_counts
    g.step(steps)
    out = [*g.params(), *g.moments(), np.asarray(g.block_deviance(steps)),
           np.asarray(g.deviance()), g.row_deviance()]
    g.close()
    return flag, out


def _same(a, b):
    for x, y in zip(a, b):
        if x is None or y is None:
            assert x is None and y is None
            continue
        assert np.array_equal(np.asarray(x), np.asarray(y))


@pytest.mark.parametrize("precision", ["fp32", "bf16", "bf16x3"])
@pytest.mark.parametrize("family", ["negbin", "poisson"])
def test_compact_counts_give_the_same_bits(precision, family):
    # 3 x 2 blocks of 766-767 rows x 350 columns (ragged row ranges and strips)
    pr = gen_nb(n=2300, m=700, d=6, R=3, S=2, seed=1961, family=family)
    steps = 2 * 6 + 3
    print(f"[case] compact counts {family} {precision}", flush=True)
    f1, a = _run(pr, precision, 1, steps)
    f0, b = _run(pr, precision, 0, steps)
    assert f1 and not f0
    _same(a, b)


def test_compact_counts_with_weights():
    pr = gen_nb(n=1500, m=520, d=4, R=2, S=3, seed=1962)
    W = np.random.default_rng(1963).uniform(0.25, 2.0, size=pr.Y.shape).astype(np.float32)
    pr = dataclasses.replace(pr, W=W)
    print("[case] compact counts with weights", flush=True)
    f1, a = _run(pr, "fp32", 1, 11)
    f0, b = _run(pr, "fp32", 0, 11)
    assert f1 and not f0
    _same(a, b)


def test_counts_that_do_not_fit_keep_float32():
    pr = gen_nb(n=900, m=400, d=3, R=2, S=2, seed=1964)
    Y = np.array(pr.Y, copy=True)
    Y[17, 33] = 70000
    pr = dataclasses.replace(pr, Y=Y)
    print("[case] compact counts: a count above 65535", flush=True)
    f1, a = _run(pr, "bf16", 1, 6)
    f0, b = _run(pr, "bf16", 0, 6)
    assert not f1 and not f0
    _same(a, b)


def test_real_valued_families_keep_float32():
    pr = gen_gaussian_lowrank(n=300, m=200, d=3, R=2, S=2)
    print("[case] compact counts: Gaussian", flush=True)
    g = gpu_for(pr, compact_counts=1)
    assert not g.compact_counts
    g.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_projection_with_compact_counts_gives_the_same_bits(precision):
    from synth import gen_nb_rows
    pr = gen_nb(n=1200, m=450, d=4, R=2, S=3, seed=1965)
    Ynew, Xnew, _, _ = gen_nb_rows(pr, 2100, seed=1966)
    A0 = np.zeros((len(Ynew), pr.q), np.float32)
    U0 = np.random.default_rng(1967).normal(0.0, 0.1, size=(len(Ynew), pr.d)).astype(np.float32)
    print(f"[case] projection with compact counts {precision}", flush=True)
    outs = []
    for compact in (1, 0):
        g = gpu_for(pr, precision=precision, compact_counts=compact)
        g.step(12)
        A, U, tr = g.project(Ynew, Xnew, A0, U0, 3, frozen=1, trace=True)
        outs.append([A.cpu().numpy(), U.cpu().numpy(), np.asarray(tr)])
        g.close()
    _same(outs[0], outs[1])
