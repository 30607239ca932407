"""Batched fits (gmf_batch_*): several contexts of different shapes and
families advanced together must follow exactly the trajectories they follow on
their own (same kernels' arithmetic, same step order per fit), with and without
the recorded HIP graph, across step-table refills; one fit is also checked
against the oracle."""
import numpy as np
import pytest

from synth import gen_nb, gen_poisson_small

from tests.gpu_helpers import compare_state, gpu_for, oracle_for, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def problems():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return [
        gen_nb(n=1800, m=900, d=7, R=4, S=3, seed=1301),                  # k = 11
        gen_poisson_small(n=700, m=500, d=12, R=5, S=2, seed=1302),       # k = 14
        gen_nb(n=2500, m=640, d=20, R=6, S=5, seed=1303, family="poisson"),  # k = 24
        gen_nb(n=333, m=1111, d=3, R=3, S=4, seed=1304),                  # ragged, k = 7
    ]


def _make(problems, stride, **over):
    return [gpu_for(pr, panel_stride=stride, skip_block_deviance=1, **over) for pr in problems]


def _state(g):
    return [np.asarray(x) for x in g.params()] + [np.asarray(x) for x in g.moments()]


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_batch_equals_separate_fits(problems, mode):
    from paper_2412_20509_amd.gmf import Batch
    print(f"[case] batch of 4 fits, mode={mode}", flush=True)
    solo = _make(problems, 32)
    for g, pr in zip(solo, problems):
        g.step(2 * pr.R * pr.S)
    fits = _make(problems, 32)
    b = Batch(fits, table_epochs=4, mode=mode)
    tr = b.run(2, eval_every=1, trace=True)
    for g, h, pr in zip(fits, solo, problems):
        assert g.steps_done() == 2 * pr.R * pr.S
        for x, y in zip(_state(g), _state(h)):
            assert np.array_equal(x, y)
    # the deviance trace is the full deviance of each fit after each epoch
    for f, (g, h) in enumerate(zip(fits, solo)):
        assert tr.shape == (4, 2)
        assert abs(tr[f, 1] - h.deviance()[0]) <= 1e-12 * abs(tr[f, 1])
    b.close()
    for g in fits + solo:
        g.close()


@pytest.mark.parametrize("precision", ["bf16", "bf16x3"])
def test_bfloat16_batch_equals_separate_fits(problems, precision):
    """The bfloat16 step tiles in a batch (level placement): the same bits as
    the fits stepped on their own (which read the 16-bit counts and run the
    8-wavefront tile in their one-step launches)."""
    from paper_2412_20509_amd.gmf import Batch
    print(f"[case] batch of 4 fits, {precision}, mode=2", flush=True)
    solo = _make(problems, 32, precision=precision)
    for g, pr in zip(solo, problems):
        g.step(2 * pr.R * pr.S)
    fits = _make(problems, 32, precision=precision)
    b = Batch(fits, table_epochs=4, mode=2)
    b.run(2, trace=False)
    for g, h, pr in zip(fits, solo, problems):
        assert g.steps_done() == 2 * pr.R * pr.S
        for x, y in zip(_state(g), _state(h)):
            assert np.array_equal(x, y)
    b.close()
    for g in fits + solo:
        g.close()


@pytest.mark.parametrize("mode", [1, 2])
def test_batch_table_refill_and_continuation(problems, mode):
    """Three epochs through a 2-epoch table, then two more epochs in a second
    call, equal five epochs stepped separately."""
    from paper_2412_20509_amd.gmf import Batch
    print(f"[case] batch refill + continuation, mode={mode}", flush=True)
    solo = _make(problems[:3], 32)
    for g, pr in zip(solo, problems):
        g.step(5 * pr.R * pr.S)
    fits = _make(problems[:3], 32)
    b = Batch(fits, table_epochs=2, mode=mode)
    b.run(3, trace=False)
    b.run(2, eval_every=2, trace=True)
    for g, h in zip(fits, solo):
        for x, y in zip(_state(g), _state(h)):
            assert np.array_equal(x, y)
    b.close()
    for g in fits + solo:
        g.close()


def test_batch_fit_matches_oracle(problems):
    from paper_2412_20509_amd.gmf import Batch
    print("[case] batch fit vs oracle", flush=True)
    pr = problems[0]
    fits = _make(problems[:2], 32)
    b = Batch(fits, table_epochs=1, use_graph=True)
    b.run(1, trace=False)
    o = oracle_for(pr)
    o.steps(pr.R * pr.S)
    compare_state(fits[0], o, 1e-5, "batched NB fit, one epoch")
    b.close()
    for g in fits:
        g.close()


def test_batch_rejects_mixed_panel_strides(problems):
    from paper_2412_20509_amd.gmf import Batch, GMFError
    fits = [gpu_for(problems[0], panel_stride=16), gpu_for(problems[1], panel_stride=32)]
    with pytest.raises(GMFError):
        Batch(fits)
    for g in fits:
        g.close()


def test_tune_records_fastest_candidate_and_plans_with_it():
    from paper_2412_20509_amd import gmf as M
    print("[case] gmf_tune on NB 3000x800", flush=True)
    pr = gen_nb(n=3000, m=800, d=6, R=3, S=2, seed=1401)
    fc = M.FitConfig(family=pr.family, d=pr.d, R=pr.R, S=pr.S, nb_alpha=pr.nb_alpha,
                     seed=pr.sched_seed)
    M.tune_table_clear()
    best, us = M.tune(fc, pr.Y, pr.X, pr.Z, pr.B0, pr.A0, pr.U0, pr.V0,
                      candidates=(32, 96, 256), steps=12)
    assert best in (32, 96, 256)
    assert all(v > 0 for v in us.values()) and us[best] == min(us.values())
    assert M.tune_lookup(fc.to_c(pr.n, pr.m, pr.p, pr.q)) == best
    # a context with tile_rows = 0 now plans with the tuned rows: same trajectory
    # as one given tile_rows = best explicitly
    g0 = gpu_for(pr)
    g1 = gpu_for(pr, tile_rows=best)
    g0.step(9)
    g1.step(9)
    for x, y in zip(_state(g0), _state(g1)):
        assert np.array_equal(x, y)
    M.tune_table_clear()
    g0.close()
    g1.close()


def test_block_deviance_of_batched_steps_is_an_error(problems):
    """gmf_batch_run forms no block deviance: asking for the block deviance of
    a batched step is an argument error, while steps run on their own after
    the batch report theirs."""
    from paper_2412_20509_amd.gmf import Batch, GMFError
    print("[case] block deviance after a batched epoch", flush=True)
    pr = problems[0]
    g = gpu_for(pr, panel_stride=32)
    b = Batch([g], table_epochs=1, use_graph=False)
    b.run(1, trace=False)
    b.close()
    with pytest.raises(GMFError):
        g.block_deviance(1)
    g.step(3)
    assert len(g.block_deviance(3)) == 3
    with pytest.raises(GMFError):
        g.block_deviance(4)
    g.close()
