"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (norm-wise relative error, max|x - ref| / max|ref|):
  * FP32 path, one step from an identical state: 1e-5 on every output array
    (parameters, the four moment arrays, the block deviance).
  * FP32 path, trajectories of many steps: 2e-4 (float32 rounding of the
    parameters compounds through the iteration).
  * Full deviance of a fixed state: 1e-6 (float32 per-entry deviance,
    float64 sums).
  * Final deviance after several epochs: 1e-4.
  * BF16 path (plain bfloat16 operands): reported only.  Its per-output
    errors and its final deviance are printed and bounded loosely (5e-2 and
    1e-3) so that a broken kernel still fails; it does not carry the 1e-4
    final-deviance target, which split BF16 meets (see test_gpu_parity_fit).
  * Split BF16 path (BF16X3): every operand keeps about 16 mantissa bits
    (|x - hi - lo| <= 2^-18 |x|) and only the lo*lo product is dropped, so a
    product is off by at most about 2^-17 relative, 128 times float32's
    operand rounding.  Parameters after one step: 1e-4 (10x the FP32 gate).
    Moments: the gradient sums cancel (signed D1), so their error is relative
    to sum |D1 P|, which exceeds max |G| by about sqrt(K) for K summed
    entries (16 at K = 260): 5e-4.  One epoch: 2e-3 (10x the FP32 trajectory
    gate).  Final deviance after several epochs: 1e-4, as for FP32.
"""
import sys

import numpy as np
import pytest

from oracle import gmf_oracle as G
from synth import gen_gaussian_lowrank, gen_nb, gen_poisson_small, gen_tiny

from tests.gpu_helpers import compare_state, gpu_for, oracle_for, rel_err

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_20509_amd import gmf  # noqa: F401  raises if libgmf.so is missing


def _one_step_case(pr, **over):
    o = oracle_for(pr, **over)
    g = gpu_for(pr, **over)
    dev_o = o.step()
    g.step(1)
    dev_g = g.block_deviance(1)[0]
    errs = compare_state(g, o, 1e-5, pr.name)
    assert rel_err([dev_g], [dev_o]) <= 1e-5, (dev_g, dev_o)
    g.close()
    return errs


def test_first_step_poisson_c1():
    pr = gen_poisson_small()
    say("first step poisson c1 1000x500 d5")
    _one_step_case(pr)


@pytest.mark.parametrize("family", ["poisson", "negbin", "gaussian"])
def test_first_step_tiny_with_covariates_and_weights(family):
    pr = gen_tiny(family, n=37, m=23, d=3, p=2, q=2, R=4, S=3, weights=True)
    say(f"first step tiny {family} 37x23 weights")
    _one_step_case(pr, lam=(0.2, 0.3, 0.7, 0.5))


@pytest.mark.parametrize("n,m,d,p,q,R,S", [
    (1000, 700, 5, 1, 1, 3, 2),      # several row ranges and a ragged column strip
    (517, 389, 12, 3, 1, 2, 3),      # KP 16, ragged everything
    (300, 260, 30, 3, 1, 2, 2),      # k = 34 -> KP 48
    (260, 200, 58, 3, 1, 2, 2),      # k = 62 -> KP 64
    (130, 90, 4, 0, 0, 1, 1),        # no covariates, full batch
])
def test_first_step_shapes(n, m, d, p, q, R, S):
    pr = gen_tiny("negbin", n=n, m=m, d=d, p=max(p, 1), q=max(q, 1), R=R, S=S, seed=1021)
    if p == 0:
        pr.p = pr.q = 0
        pr.X = np.zeros((n, 0)); pr.Z = np.zeros((m, 0))
        pr.B0 = np.zeros((m, 0)); pr.A0 = np.zeros((n, 0))
    say(f"first step shape n={n} m={m} d={d} p={p} q={q} R={R} S={S}")
    _one_step_case(pr)


def test_trajectory_one_epoch_c1():
    pr = gen_poisson_small()
    say("trajectory c1 one epoch")
    o = oracle_for(pr)
    g = gpu_for(pr)
    devs_o = o.epoch()
    g.step(pr.R * pr.S)
    devs_g = g.block_deviance(pr.R * pr.S)
    compare_state(g, o, 2e-4, "c1 epoch")
    assert rel_err(devs_g, devs_o) <= 1e-4
    g.close()


def test_trajectory_nb_covariates():
    pr = gen_nb(n=2000, m=800, d=6, R=4, S=4, seed=1031)
    say("trajectory nb 2000x800 d6 covariates, 40 steps")
    o = oracle_for(pr)
    g = gpu_for(pr)
    o.steps(40)
    g.step(40)
    compare_state(g, o, 2e-4, "nb trajectory")
    g.close()


def test_schedule_of_context_matches_oracle():
    pr = gen_poisson_small(n=300, m=200, R=7, S=3)
    say("schedule from context")
    g = gpu_for(pr)
    rp, cp, rr = g.schedule(1, 100)
    o = oracle_for(pr)
    assert np.array_equal(rp, o.row_perm)
    assert np.array_equal(cp, o.col_perm)
    assert rr.tolist() == [o.block_of_step(t)[0] for t in range(1, 101)]
    g.close()


def test_full_deviance_matches_oracle():
    for pr in (gen_poisson_small(), gen_nb(n=1500, m=700, d=5, R=3, S=2, seed=1032),
               gen_tiny("gaussian", n=200, m=130, d=4, p=2, q=1, R=2, S=2, weights=True)):
        say(f"full deviance {pr.name}")
        o = oracle_for(pr)
        g = gpu_for(pr)
        dg, pg = g.deviance()
        assert rel_err([dg], [o.full_deviance()]) <= 1e-6, (dg, o.full_deviance())
        assert rel_err([pg], [o.objective()]) <= 1e-6
        g.close()


@pytest.mark.parametrize("family,weights,d", [("negbin", False, 6), ("poisson", True, 6),
                                              ("gaussian", True, 4), ("negbin", False, 40)])
def test_row_deviance_matches_oracle(family, weights, d):
    """gmf_row_deviance against the oracle's per-row deviance of the same
    parameters, and its rows add up to gmf_deviance's total (1e-6: float32
    entries, different order).  Per row the float32 error of eta grows with
    the number of its products K = p + q + d (the deviance's dependence on eta
    carries it): 1e-6 norm-relative at K <= 16, as for the full deviance, and
    1e-6 K / 16 rounded up to 4e-6 at K = 44."""
    pr = gen_tiny(family, n=700, m=530, d=d, p=2, q=2, R=3, S=4, weights=weights, seed=1801)
    say(f"row deviance {family} d={d} weights={weights}")
    o = oracle_for(pr)
    g = gpu_for(pr)
    g.step(10)
    B, A, U, V = g.params()
    ref = G.row_deviance(o.cfg, pr.Y, pr.X, pr.Z, B, A, U, V, W=pr.W)
    rows = g.row_deviance()
    total, _ = g.deviance()
    print("row deviance error", rel_err(rows, ref), "sum vs total", abs(rows.sum() - total) / total)
    assert rows.shape == (pr.n,)
    k = pr.p + pr.q + pr.d
    assert rel_err(rows, ref) <= (1e-6 if k <= 16 else 4e-6)
    assert abs(rows.sum() - total) <= 1e-6 * abs(total)
    g.close()


def test_final_deviance_after_epochs_c1():
    pr = gen_poisson_small()
    say("final deviance c1 after 20 epochs")
    o = oracle_for(pr)
    g = gpu_for(pr)
    for _ in range(20):
        o.epoch()
    rc, trace, done = g.fit(20, 0.0, 5)
    assert done == 20 and len(trace) == 4
    d_o = o.full_deviance()
    assert abs(trace[-1] - d_o) / d_o <= 1e-4, (trace[-1], d_o)
    g.close()


def test_steps_are_deterministic():
    pr = gen_nb(n=1200, m=600, d=8, R=3, S=3, seed=1033)
    say("determinism")
    outs = []
    for _ in range(2):
        g = gpu_for(pr)
        g.step(25)
        outs.append(g.params())
        g.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "bf16x3"])
def test_steps_are_deterministic_under_load(precision):
    """Two runs of the same fit, with many workgroups per compute unit and
    many 32-row groups per tile (blocks of 5000 x 1000): every parameter,
    moment, block deviance and the full deviance the same bits.  Tolerance
    tests cannot see a race between the wavefronts of a tile; this one can."""
    pr = gen_nb(n=20000, m=3000, d=20, R=4, S=3, seed=1035)
    say(f"determinism under load, {precision}")
    outs = []
    for _ in range(2):
        g = gpu_for(pr, precision=precision)
        g.step(24)
        outs.append([*g.params(), *g.moments(), np.asarray(g.block_deviance(24)),
                     np.asarray(g.deviance())])
        g.close()
    for a, b in zip(*outs):
        assert np.array_equal(np.asarray(a), np.asarray(b))


def test_postprocess_matches_oracle_projection():
    pr = gen_nb(n=900, m=400, d=5, R=3, S=2, seed=1034)
    say("postprocess A+B1")
    g = gpu_for(pr)
    g.step(30)
    B, A, U, V = g.params(0)
    Bp, Ap, Up, Vp = g.params(1)
    rB, rA, rU, rV = G.postprocess_A_B1(pr.X, pr.Z, B, A, U, V)
    for name, x, ref in (("B", Bp, rB), ("Gamma", Ap, rA), ("U", Up, rU), ("V", Vp, rV)):
        assert rel_err(x, ref) <= 2e-5, (name, rel_err(x, ref))
    # invariants hold on the device result too
    eta = pr.X @ B.T + A @ pr.Z.T + U @ V.T
    eta_p = pr.X @ Bp.T + Ap @ pr.Z.T + Up @ Vp.T
    assert rel_err(eta_p, eta) <= 2e-5
    np.testing.assert_allclose(Vp.T @ Vp, np.eye(pr.d), atol=2e-5)
    g.close()


def test_bf16_path_reports_errors():
    """Plain BF16, reported only: per-output errors after one epoch and the
    final deviance after 20 epochs, with loose sanity bounds."""
    pr = gen_poisson_small()
    say("bf16 c1 (reported only): per-output errors after one epoch, final deviance after 20 epochs")
    o = oracle_for(pr)
    g = gpu_for(pr, precision="bf16")
    o.epoch()
    g.step(pr.R * pr.S)
    B, A, U, V = g.params()
    errs = {"B": rel_err(B, o.B), "Gamma": rel_err(A, o.A), "U": rel_err(U, o.U),
            "V": rel_err(V, o.V)}
    print("bf16 one-epoch relative errors:", errs)
    assert max(errs.values()) < 5e-2
    for _ in range(19):
        o.epoch()
    g.step(19 * pr.R * pr.S)
    dg, _ = g.deviance()
    d_o = o.full_deviance()
    print("bf16 final deviance rel err:", abs(dg - d_o) / d_o)
    assert abs(dg - d_o) / d_o <= 1e-3
    g.close()


def test_error_paths():
    from paper_2412_20509_amd.gmf import GMFError, GMF_ENUMERIC, GMF_EINVAL
    pr = gen_tiny("poisson", n=40, m=30, d=2, R=2, S=2)
    say("error paths")
    bad = pr.Y.copy()
    bad[3, 4] = -1
    pr2 = gen_tiny("poisson", n=40, m=30, d=2, R=2, S=2)
    pr2.Y = bad
    with pytest.raises(GMFError) as ei:
        gpu_for(pr2)
    assert ei.value.code == GMF_EINVAL
    g = gpu_for(pr, rate0=1e38, decay=0.0, damping=0.0)
    g.step(3)
    with pytest.raises(GMFError) as ei:
        g.sync()
    assert ei.value.code == GMF_ENUMERIC
    g.close()


def test_gaussian_full_batch_reaches_truncated_svd():
    pr = gen_gaussian_lowrank()
    say("gaussian full batch -> truncated SVD")
    g = gpu_for(pr, lam=(0, 0, 0.5, 0.5), rate0=0.5, decay=0.0, alpha1=1.0, alpha2=1.0,
                damping=0.0)
    g.step(1500)
    _, _, U, V = g.params()
    P, s, Qt = np.linalg.svd(pr.Y, full_matrices=False)
    M = (P[:, :3] * np.maximum(s[:3] - 0.5, 0)) @ Qt[:3]
    assert np.linalg.norm(U @ V.T - M) / np.linalg.norm(M) < 1e-5
    g.close()


@pytest.mark.parametrize("overlap", [0, 1])
def test_run_with_deviance_equals_step_then_deviance(overlap):
    """gmf_run evaluates the deviance in order on the context's stream, or from
    a snapshot on a second stream; the values equal gmf_deviance after the same
    epochs, the iterate equals plain stepping, and the device completion times
    increase."""
    from synth import make_problem
    print(f"[case] gmf_run (overlap={overlap}) vs step + deviance, Poisson 1000x500", flush=True)
    pr = make_problem("c1")
    g1 = gpu_for(pr, eval_overlap=overlap)
    g2 = gpu_for(pr)
    tr, ms = g1.run(5, eval_every=2)
    ref = []
    for e in range(5):
        g2.step(pr.R * pr.S)
        if (e + 1) % 2 == 0:
            ref.append(g2.deviance()[0])
    assert len(tr) == 2 and tr == ref
    assert 0 < ms[0] < ms[1]
    for x, y in zip(g1.params() + tuple(g1.moments()), g2.params() + tuple(g2.moments())):
        assert np.array_equal(x, y)
    tr2, _ = g1.run(3, eval_every=1)            # a second call continues the fit
    for _ in range(3):
        g2.step(pr.R * pr.S)
    assert tr2[-1] == g2.deviance()[0]
    g1.close()
    g2.close()


@pytest.mark.parametrize("precision,d", [("fp32", 10), ("fp32", 20), ("bf16", 10), ("bf16x3", 10)])
def test_eight_wave_tiles_equal_four_wave_tiles(precision, d):
    """The 8-wavefront tile splits each 32-row group between two wavefronts
    but keeps every product and sum of the step in the same order: the
    iterates are bit-identical to the 4-wavefront tile's.  The block deviance
    (a monitor) sums each lane's entries in float32 before float64, over 8
    instead of 16 entries, so it agrees to float32 rounding only."""
    print(f"[case] tile waves 4 vs 8, {precision} d={d}", flush=True)
    pr = gen_nb(n=2600, m=900, d=d, R=4, S=3, seed=1500 + d)
    # bfloat16 8-wavefront tiles exist at panel stride 32
    ps = 0 if precision == "fp32" else 32
    g4 = gpu_for(pr, precision=precision, tile_waves=4, panel_stride=ps)
    g8 = gpu_for(pr, precision=precision, tile_waves=8, panel_stride=ps)
    g4.step(20)
    g8.step(20)
    for x, y in zip(g4.params() + tuple(g4.moments()), g8.params() + tuple(g8.moments())):
        assert np.array_equal(x, y)
    b4, b8 = g4.block_deviance(20), g8.block_deviance(20)
    assert np.max(np.abs(b4 - b8) / np.abs(b4)) < 1e-6
    g4.close()
    g8.close()


def test_precision_switch():
    """A BF16 context switched to FP32 steps exactly like an FP32 context of the
    same panel stride (16 here); an FP32 context at stride 48 cannot switch to
    a bfloat16 precision (its products need stride 16, 32 or 64)."""
    from paper_2412_20509_amd.gmf import GMFError
    print("[case] precision switch", flush=True)
    pr = gen_nb(n=1500, m=600, d=6, R=3, S=2, seed=1601)
    gb = gpu_for(pr, precision="bf16")                   # stride 16
    gf = gpu_for(pr, precision="fp32")                   # stride 16
    gb.set_precision("fp32")
    gb.step(12)
    gf.step(12)
    for x, y in zip(gb.params() + tuple(gb.moments()), gf.params() + tuple(gf.moments())):
        assert np.array_equal(x, y)
    pr48 = gen_nb(n=600, m=300, d=40, R=2, S=2, seed=1602)   # p + q + d = 44 -> 48
    g48 = gpu_for(pr48, precision="fp32")
    with pytest.raises(GMFError):
        g48.set_precision("bf16")
    g48.step(2)
    for g in (gb, gf, g48):
        g.close()

@pytest.mark.parametrize("family,n,m,d,R,S", [
    ("poisson", 1000, 700, 5, 3, 2),     # several row ranges and a ragged column strip
    ("negbin", 517, 389, 12, 2, 3),      # ragged everything
    ("gaussian", 300, 260, 20, 2, 2),
    ("negbin", 260, 200, 40, 2, 2),      # k = 44 -> panel stride 64
])
def test_bf16x3_first_step(family, n, m, d, R, S):
    pr = gen_tiny(family, n=n, m=m, d=d, p=2, q=2, R=R, S=S, seed=1701, weights=True)
    say(f"bf16x3 first step {family} n={n} m={m} d={d}")
    lam = (0.2, 0.3, 0.7, 0.5)
    o = oracle_for(pr, lam=lam)
    g = gpu_for(pr, precision="bf16x3", lam=lam)
    dev_o = o.step()
    g.step(1)
    errs = compare_state(g, o, 5e-4, f"bf16x3 {family}")
    print("bf16x3 one-step relative errors:", errs)
    for k in ("B", "Gamma", "U", "V"):
        assert errs[k] <= 1e-4, (k, errs[k])
    assert rel_err([g.block_deviance(1)[0]], [dev_o]) <= 1e-4
    g.close()


@pytest.mark.parametrize("family,n,m,d,R,S", [
    ("poisson", 1000, 700, 5, 3, 2),     # panel stride 16 (16x16x16 products), a ragged strip
    ("negbin", 517, 389, 20, 2, 3),      # k = 24 -> panel stride 32, ragged everything
    ("negbin", 260, 200, 40, 2, 2),      # k = 44 -> panel stride 64
])
def test_bf16_first_step(family, n, m, d, R, S):
    """Plain BF16 (bfloat16 operands in eta and in the four contractions, with
    weights) at each panel stride: one step against the oracle.  bfloat16
    keeps 8 bits of each operand (relative rounding up to 2^-9); measured on
    these cases: parameters within 8.3e-4, moments within 4.2e-3 (the
    curvature sums of squared operands round the most), the block deviance
    within 7.1e-5; gated at 3e-3, 1e-2 and 3e-4."""
    pr = gen_tiny(family, n=n, m=m, d=d, p=2, q=2, R=R, S=S, seed=1702, weights=True)
    say(f"bf16 first step {family} n={n} m={m} d={d}")
    lam = (0.2, 0.3, 0.7, 0.5)
    o = oracle_for(pr, lam=lam)
    g = gpu_for(pr, precision="bf16", lam=lam)
    dev_o = o.step()
    g.step(1)
    errs = compare_state(g, o, 1e-2, f"bf16 {family}")
    print("bf16 one-step relative errors:", errs)
    for k in ("B", "Gamma", "U", "V"):
        assert errs[k] <= 3e-3, (k, errs[k])
    dev_err = rel_err([g.block_deviance(1)[0]], [dev_o])
    print("bf16 block deviance relative error:", dev_err)
    assert dev_err <= 3e-4
    g.close()


def test_bf16x3_reaches_oracle_deviance():
    pr = gen_poisson_small()
    say("bf16x3 c1: one epoch, final deviance after 20 epochs")
    o = oracle_for(pr)
    g = gpu_for(pr, precision="bf16x3")
    o.epoch()
    g.step(pr.R * pr.S)
    errs = compare_state(g, o, 2e-3, "bf16x3 c1 epoch")
    print("bf16x3 one-epoch relative errors:", errs)
    for _ in range(19):
        o.epoch()
    g.step(19 * pr.R * pr.S)
    dg, _ = g.deviance()
    d_o = o.full_deviance()
    print("bf16x3 final deviance rel err:", abs(dg - d_o) / d_o)
    assert abs(dg - d_o) / d_o <= 1e-4
    g.close()
