"""Parity at the full size of the large workload: NB(alpha=5) 100,000 x 5,000,
rank 20, X = [1, batch, N(0,1)], Z = 1, blocks 10,000 x 1,000 (R = 10, S = 5),
in the launch configuration the benchmark times.

The oracle runs the same first steps in FP64 (a block step is cheap for it);
every output array is compared element by element: 1e-5 relative for the FP32
path, and the BF16 path's errors are reported per output with a loose gate.
"""
import sys

import numpy as np
import pytest

from oracle import gmf_oracle as G
from synth import make_problem

from tests.gpu_helpers import compare_state, gpu_for, oracle_for, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c3():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[case] generating NB 100000x5000 d20", flush=True)
    return make_problem("c3")


def test_large_first_steps_fp32(c3):
    print("[case] large fp32: 2 steps vs oracle", flush=True)
    o = oracle_for(c3)
    g = gpu_for(c3)
    dev_o = o.steps(2)
    g.step(2)
    dev_g = g.block_deviance(2)
    compare_state(g, o, 1e-5, "NB 100000x5000 fp32, 2 steps")
    assert rel_err(dev_g, dev_o) <= 1e-5
    g.close()


def test_large_first_step_bf16_errors(c3):
    print("[case] large bf16: 1 step vs oracle", flush=True)
    o = oracle_for(c3)
    g = gpu_for(c3, precision="bf16")
    o.step()
    g.step(1)
    B, A, U, V = g.params()
    Gr, Hr, Gc, Hc = g.moments()
    errs = {"B": rel_err(B, o.B), "Gamma": rel_err(A, o.A), "U": rel_err(U, o.U),
            "V": rel_err(V, o.V), "Grow": rel_err(Gr, o.Grow), "Hrow": rel_err(Hr, o.Hrow),
            "Gcol": rel_err(Gc, o.Gcol), "Hcol": rel_err(Hc, o.Hcol)}
    print("bf16 per-output relative errors after one step:", errs, flush=True)
    sys.stdout.flush()
    assert max(errs.values()) < 3e-2
    g.close()


def test_large_first_step_bf16x3(c3):
    """Split BF16 at full size (panel stride 32, 16x16x32 products): one step,
    the same gates as the small split-BF16 cases (parameters 1e-4, moments
    5e-4, block deviance 1e-4)."""
    print("[case] large bf16x3: 1 step vs oracle", flush=True)
    o = oracle_for(c3)
    g = gpu_for(c3, precision="bf16x3")
    dev_o = o.step()
    g.step(1)
    errs = compare_state(g, o, 5e-4, "NB 100000x5000 bf16x3, 1 step")
    print("bf16x3 per-output relative errors after one step:", errs, flush=True)
    for k in ("B", "Gamma", "U", "V"):
        assert errs[k] <= 1e-4, (k, errs[k])
    assert rel_err([g.block_deviance(1)[0]], [dev_o]) <= 1e-4
    g.close()


def test_large_row_deviance_sampled(c3):
    """gmf_row_deviance at full size after one epoch in the benchmark's launch
    configuration: 2,000 sampled rows against the oracle's per-row deviance of
    the same parameters (gate 1e-6 K/16 for K = p + q + d = 24 products in
    eta, times 2), and all rows add up to gmf_deviance's total."""
    print("[case] large row deviance: one epoch, 2000 sampled rows", flush=True)
    o = oracle_for(c3)
    g = gpu_for(c3)
    g.step(c3.R * c3.S)
    B, A, U, V = g.params()
    rows = g.row_deviance()
    total, _ = g.deviance()
    idx = np.sort(np.random.default_rng(5).choice(c3.n, 2000, replace=False))
    ref = G.row_deviance(o.cfg, c3.Y[idx], c3.X[idx], c3.Z, B, A[idx], U[idx], V)
    err = rel_err(rows[idx], ref)
    print("sampled row deviance error", err, "sum vs total", abs(rows.sum() - total) / total,
          flush=True)
    assert rows.shape == (c3.n,)
    assert err <= 3e-6
    assert abs(rows.sum() - total) <= 1e-6 * abs(total)
    g.close()
