"""Parity of whole fits and of the less common step options with the oracle.

  * The 10000 x 2000 NB(alpha = 5) fit, 200 epochs through gmf_run (the
    deviance of every epoch evaluated on the device), against the oracle's
    deviance after every epoch of the same seeded schedule
    (tests/golden/oracle_trace_c2.json, written by make_golden.py from the
    oracle alone): within 1e-4 relative at every epoch in FP32 and in split
    BF16 (the arm that carries the bfloat16 claim).  Plain BF16 is reported
    only (its rounding of D1/D2 and the panels delays the iteration; its
    distance to the oracle is printed and bounded loosely).
  * The printed bias factor of eq. 11 (bias_mode = 1): one step at 1e-5 and
    one epoch at 2e-4, the FP32 tolerances.
  * The clamp of the log link (eta in [log eps, eta_max]): starting values
    that put eta above 30 on some entries and below log 1e-8 on others; one
    step at 1e-5.
"""
import json
import os
import sys

import numpy as np
import pytest

from synth import gen_poisson_small, gen_tiny, make_problem

from tests.gpu_helpers import compare_state, gpu_for, oracle_for, rel_err

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_20509_amd import gmf  # noqa: F401  raises if libgmf.so is missing


@pytest.fixture(scope="module")
def c2_problem():
    return make_problem("c2")


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "bf16"])
def test_c2_fit_tracks_oracle_trace_every_epoch(c2_problem, precision):
    tr = json.load(open(os.path.join(GOLDEN, "oracle_trace_c2.json")))
    ref = np.asarray(tr["deviance_per_epoch"], np.float64)
    epochs = tr["epochs"]
    pr = c2_problem
    say(f"c2 10000x2000 NB d=10, {epochs} epochs, {precision}, vs oracle trace")
    g = gpu_for(pr, precision=precision, rate0=tr["rate0"], decay=tr["decay"], tau=tr["tau"],
                alpha1=tr["alpha1"], alpha2=tr["alpha2"], damping=tr["damping"],
                lam=tr["lam"])
    d0, _ = g.deviance()
    assert rel_err([d0], [ref[0]]) <= 1e-6
    devs, _ = g.run(epochs, eval_every=1)
    devs = np.asarray(devs)
    rel = np.abs(devs - ref[1:]) / ref[1:]
    print(f"{precision}: max rel. deviation from the oracle over {epochs} epochs "
          f"{rel.max():.3e} (epoch {int(rel.argmax()) + 1}), final {rel[-1]:.3e}")
    if precision == "bf16":
        # reported only: plain bfloat16 trails the iteration (about 1e-3 at the end)
        assert rel[-1] < 3e-3
    else:
        assert rel.max() <= 1e-4
    g.close()


@pytest.mark.parametrize("precision", ["bf16", "bf16x3"])
def test_bfloat16_arms_reach_oracle_final_deviance(c2_problem, precision):
    """The spec claim for the bfloat16 arms: continued past the oracle's
    200-epoch budget (to 300 epochs), the fit comes within 1e-4 of D* (the
    oracle's deviance after 200 epochs) -- plain BF16 trails the FP32
    trajectory by about 1e-3 at epoch 200 and catches up about 20 epochs
    later -- and stays below D* (1 + 1e-4) from there on."""
    tr = json.load(open(os.path.join(GOLDEN, "oracle_trace_c2.json")))
    dstar = tr["final"]
    pr = c2_problem
    say(f"c2 {precision}, 300 epochs, first epoch within 1e-4 of the oracle's D*")
    g = gpu_for(pr, precision=precision, rate0=tr["rate0"], decay=tr["decay"], tau=tr["tau"],
                alpha1=tr["alpha1"], alpha2=tr["alpha2"], damping=tr["damping"],
                lam=tr["lam"])
    devs, _ = g.run(300, eval_every=1)
    devs = np.asarray(devs)
    hit = np.nonzero(np.abs(devs - dstar) <= 1e-4 * dstar)[0]
    print(f"{precision}: first epoch within 1e-4 of D*: {hit[0] + 1 if len(hit) else None}, "
          f"epoch 300 {(devs[-1] - dstar) / dstar:+.3e}")
    assert len(hit) > 0 and hit[0] + 1 <= 260
    assert np.all(devs[hit[0]:] <= dstar * (1 + 1e-4))
    g.close()


def test_bias_mode_printed_formula_one_step_and_epoch():
    pr = gen_poisson_small()
    say("bias_mode = 1 (printed alpha_t): one step, one epoch, c1")
    o = oracle_for(pr, bias_mode=1)
    g = gpu_for(pr, bias_mode=1)
    dev_o = o.step()
    g.step(1)
    compare_state(g, o, 1e-5, "bias_mode 1, one step")
    assert rel_err([g.block_deviance(1)[0]], [dev_o]) <= 1e-5
    o.steps(pr.R * pr.S - 1)
    g.step(pr.R * pr.S - 1)
    compare_state(g, o, 2e-4, "bias_mode 1, one epoch")
    g.close()


@pytest.mark.parametrize("family", ["poisson", "negbin"])
def test_clamped_entries_one_step(family):
    """Rows whose intercept puts eta above eta_max = 30 on some entries (row 0:
    gamma 31 with u'v spread over +-2) and below log 1e-8 on others (row 1:
    gamma -19.5, row 2 straddles both bounds through a large u)."""
    pr = gen_tiny(family, n=150, m=120, d=3, p=2, q=1, R=2, S=2, seed=1901)
    A0 = pr.A0.copy()
    U0 = pr.U0.copy()
    A0[0, 0] = 31.0
    A0[1, 0] = -19.5
    U0[2] = [60.0, 0.0, 0.0]
    pr.A0 = A0.astype(np.float32).astype(np.float64)
    pr.U0 = U0.astype(np.float32).astype(np.float64)
    eta = pr.X @ pr.B0.T + pr.A0 @ pr.Z.T + pr.U0 @ pr.V0.T
    hi, lo = int((eta > 30).sum()), int((eta < np.log(1e-8)).sum())
    say(f"clamp one step {family}: {hi} entries above 30, {lo} below log 1e-8")
    assert hi >= 20 and lo >= 20
    # every row block is drawn within a few steps; run until rows 0-2 were touched
    o = oracle_for(pr)
    g = gpu_for(pr)
    for t in range(4):
        dev_o = o.step()
        g.step(1)
        compare_state(g, o, 1e-5, f"clamp {family} step {t + 1}")
        assert rel_err([g.block_deviance(1)[0]], [dev_o]) <= 1e-5
    g.close()
