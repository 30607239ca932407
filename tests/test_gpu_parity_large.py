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
