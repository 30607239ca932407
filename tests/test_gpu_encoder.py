"""Parity of the warm-start encoder (gmf_encoder_*) with the FP64 MLP oracle.

Sizes: m = 300 inputs (9 K-steps of 32 and a ragged 12), hidden = 96 (one full
and one ragged 64-wide tile), d = 5, minibatch 48 (a ragged row tile), and a
200-row epoch whose last minibatch holds 8 rows.  The float32 path must agree
with the oracle to float32 accumulation error; the bfloat16 inference path is
held to the bfloat16 operand rounding it introduces.
"""
import numpy as np
import pytest

from synth import gen_nb_rows, make_problem, mlp_init
from oracle.mlp_oracle import MLP, PARAM_NAMES

pytestmark = pytest.mark.gpu

M, H, D, BATCH = 300, 96, 5, 48


def nrel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def data():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(4242)
    lam = rng.gamma(0.6, 2.0, size=(200, M))
    Y = rng.poisson(lam).astype(np.int32)
    U = rng.standard_normal((200, D)).astype(np.float32)
    w = mlp_init(M, H, D, seed=99)
    return Y, U, w


def make_encoder(w, **kw):
    from paper_2412_20509_amd.gmf import Encoder
    kw.setdefault("hidden", H)
    kw.setdefault("batch", BATCH)
    return Encoder(M, D, w, **kw)


def oracle_mlp(w):
    return MLP(*(np.asarray(w[k], np.float64) for k in PARAM_NAMES))


def test_loss_and_gradients_match_oracle(data):
    Y, U, w = data
    print("[case] encoder loss/grad m300 h96 d5 rows48", flush=True)
    enc = make_encoder(w)
    loss_g, grads_g = enc.loss_grad(Y[:BATCH], U[:BATCH])
    loss_o, grads_o = oracle_mlp(w).loss_and_grads(Y[:BATCH], U[:BATCH].astype(np.float64))
    assert abs(loss_g - loss_o) <= 1e-5 * loss_o
    for k in PARAM_NAMES:
        assert grads_g[k].shape == grads_o[k].shape, k
        assert nrel(grads_g[k], grads_o[k]) <= 1e-4, (k, nrel(grads_g[k], grads_o[k]))
    enc.close()


def test_ragged_batch_gradients(data):
    Y, U, w = data
    print("[case] encoder loss/grad 7 rows", flush=True)
    enc = make_encoder(w)
    loss_g, grads_g = enc.loss_grad(Y[5:12], U[5:12])
    loss_o, grads_o = oracle_mlp(w).loss_and_grads(Y[5:12], U[5:12].astype(np.float64))
    assert abs(loss_g - loss_o) <= 1e-5 * loss_o
    for k in PARAM_NAMES:
        assert nrel(grads_g[k], grads_o[k]) <= 1e-4, k
    enc.close()


def test_adam_epoch_matches_oracle(data):
    """One epoch of 5 Adam steps (last minibatch ragged): the per-epoch loss and
    every weight update agree with the oracle."""
    Y, U, w = data
    print("[case] encoder 1 epoch Adam vs oracle", flush=True)
    enc = make_encoder(w, lr=1e-3, weight_decay=1e-2)
    tr_g = enc.train(Y, U, 1)
    wg = enc.weights()
    o = oracle_mlp(w)
    tr_o = o.train(Y, U.astype(np.float64), 1, BATCH, 1e-3, wd=1e-2)
    assert abs(tr_g[0] - tr_o[0]) <= 1e-5 * tr_o[0]
    for k in PARAM_NAMES:
        dg = wg[k] - w[k]
        do = getattr(o, k) - w[k]
        # Adam's normalised step is sign-like where a gradient is near zero, so
        # compare the updates as a whole rather than element by element.
        assert nrel(dg, do) <= 5e-3, (k, nrel(dg, do))
    enc.close()


def test_training_reduces_loss(data):
    Y, U, w = data
    print("[case] encoder 40 epochs, loss decreases", flush=True)
    # a learnable target: the output of another network of the same shape
    teacher = oracle_mlp(mlp_init(M, H, D, seed=7))
    T = teacher.forward(Y)[0].astype(np.float32)
    enc = make_encoder(w, lr=3e-3)
    tr = enc.train(Y, T, 40)
    assert all(np.isfinite(tr))
    assert tr[-1] < 0.3 * tr[0], tr


def test_forward_fp32_matches_oracle_and_bf16_close(data):
    Y, U, w = data
    print("[case] encoder forward fp32/bf16 200 rows", flush=True)
    enc = make_encoder(w)
    out_o = oracle_mlp(w).forward(Y)[0]
    f32 = enc.forward(Y, bf16=False).cpu().numpy()
    b16 = enc.forward(Y, bf16=True).cpu().numpy()
    assert nrel(f32, out_o) <= 1e-5
    assert nrel(b16, out_o) <= 2e-2
    # counts given as float32 values read the same
    f32b = enc.forward(Y.astype(np.float32), bf16=False).cpu().numpy()
    assert np.array_equal(f32, f32b)
    enc.close()


def test_forward_many_rows_default_width():
    """More rows than one inference chunk (65,536), hidden 256, the NB workload's
    column count; sampled rows against the oracle."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[case] encoder forward 70000 x 2000 rows, hidden 256", flush=True)
    pr = make_problem("c2")
    Ynew = gen_nb_rows(pr, 70000, seed=5)[0]
    w = mlp_init(pr.m, 256, pr.d, seed=3)
    from paper_2412_20509_amd.gmf import Encoder
    enc = Encoder(pr.m, pr.d, w, hidden=256, batch=256)
    f32 = enc.forward(Ynew, bf16=False).cpu().numpy()
    b16 = enc.forward(Ynew, bf16=True).cpu().numpy()
    rows = np.r_[0:3, 65533:65539, 69997:70000]
    out_o = oracle_mlp(w).forward(Ynew[rows])[0]
    assert nrel(f32[rows], out_o) <= 1e-5
    assert nrel(b16[rows], out_o) <= 2e-2
    assert np.isfinite(b16).all()
    enc.close()


def test_encoder_rejects_bad_sizes(data):
    from paper_2412_20509_amd.gmf import GMFError
    Y, U, w = data
    enc = make_encoder(w)
    with pytest.raises(GMFError):
        enc.loss_grad(Y[:BATCH + 1], U[:BATCH + 1])
    enc.close()


@pytest.mark.parametrize("hidden,d", [(64, 5), (128, 10), (256, 20)])
def test_fused_bf16_inference_equals_layer_by_layer(hidden, d):
    """The fused bfloat16 kernel (three layers per 64-row workgroup) makes the
    same products in the same order, with the same bfloat16 rounding points,
    as the layer-by-layer bfloat16 path: identical outputs, on a row count
    that leaves a ragged last workgroup and a column count with a K tail."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print(f"[case] fused vs layered bf16 inference, hidden={hidden} d={d}", flush=True)
    from paper_2412_20509_amd.gmf import Encoder
    rng = np.random.default_rng(3 + hidden)
    m = 1000                                   # 31 K-tiles of 32 and a tail of 8
    Y = rng.poisson(rng.gamma(0.5, 2.0, size=(777, m))).astype(np.int32)
    w = mlp_init(m, hidden, d, seed=hidden)
    enc = Encoder(m, d, w, hidden=hidden, batch=64)
    fused = enc.forward(Y, bf16=True, fused=True).cpu().numpy()
    layered = enc.forward(Y, bf16=True, fused=False).cpu().numpy()
    assert np.array_equal(fused, layered)
    out_o = oracle_mlp(w).forward(Y)[0]
    assert nrel(fused, out_o) <= 2e-2
    # after a training step the bfloat16 weight copies are refreshed
    enc.train(Y[:64], rng.standard_normal((64, d)).astype(np.float32), 1)
    fused2 = enc.forward(Y, bf16=True, fused=True).cpu().numpy()
    layered2 = enc.forward(Y, bf16=True, fused=False).cpu().numpy()
    assert np.array_equal(fused2, layered2) and not np.array_equal(fused2, fused)
    enc.close()
