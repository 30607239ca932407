"""Checkpoint and resume of a fit (gmf_save_state / gmf_load_state): a run
saved after k steps and resumed in a fresh context continues the seeded
schedule of Algorithm 1 exactly, bit for bit, in every precision."""
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


def _snapshot(g, nblock):
    B, A, U, V = g.params()
    return [B, A, U, V, *g.moments(), np.asarray(g.block_deviance(nblock)), g.steps_done()]


@pytest.mark.parametrize("precision", ["fp32", "bf16", "bf16x3"])
def test_resume_is_bit_identical(precision):
    pr = gen_nb(n=2100, m=650, d=5, R=4, S=3, seed=1951)
    print(f"[case] save/load state {precision}", flush=True)
    k, more = 17, 29
    g1 = gpu_for(pr, precision=precision)
    g1.step(k)
    state = g1.save_state()
    g1.step(more)
    ref = _snapshot(g1, more)
    # a fresh context of the same problem, stepped elsewhere first, then resumed
    g2 = gpu_for(pr, precision=precision)
    g2.step(5)
    g2.load_state(state)
    assert g2.steps_done() == k
    g2.step(more)
    got = _snapshot(g2, more)
    for a, b in zip(ref[:-1], got[:-1]):
        assert np.array_equal(np.asarray(a), np.asarray(b))
    assert got[-1] == ref[-1] == k + more
    # saving the resumed context reproduces the uninterrupted context's state
    assert g2.save_state() == g1.save_state()
    g1.close()
    g2.close()


def test_load_state_rejects_other_problems():
    from paper_2412_20509_amd.gmf import GMFError
    pr = gen_nb(n=800, m=300, d=4, R=2, S=3, seed=1952)
    print("[case] load_state argument checks", flush=True)
    g = gpu_for(pr)
    g.step(4)
    state = g.save_state()
    before = g.save_state()
    other_seed = gpu_for(pr, seed=pr.sched_seed + 1)
    with pytest.raises(GMFError):
        other_seed.load_state(state)
    other_rate = gpu_for(pr, rate0=0.07)
    with pytest.raises(GMFError):
        other_rate.load_state(state)
    bad = bytearray(state)
    bad[0] ^= 0xFF
    with pytest.raises(GMFError):
        g.load_state(bytes(bad))
    with pytest.raises(GMFError):
        g.load_state(state[:len(state) // 2])
    assert g.save_state() == before          # failed loads leave the context as it was
    for x in (g, other_seed, other_rate):
        x.close()
