"""Pins of the encoder oracle: GELU against the normal CDF, gradients against
finite differences, the first Adam step, and a training run that learns."""
import numpy as np
from scipy import stats

from oracle import mlp_oracle as M
from synth import mlp_init


def _tiny(seed=3):
    w = mlp_init(16, 8, 3, seed=seed)
    return M.MLP(w["W1"], w["b1"], w["W2"], w["b2"], w["W3"], w["b3"])


def test_gelu_is_z_times_normal_cdf():
    z = np.linspace(-6, 6, 101)
    np.testing.assert_allclose(M.gelu(z), z * stats.norm.cdf(z), rtol=1e-12, atol=1e-15)
    h = 1e-6
    np.testing.assert_allclose(M.gelu_grad(z), (M.gelu(z + h) - M.gelu(z - h)) / (2 * h),
                               rtol=1e-7, atol=1e-9)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    net = _tiny()
    Y = rng.poisson(1.5, size=(5, 16))
    U = rng.normal(size=(5, 3))
    _, g = net.loss_and_grads(Y, U)
    h = 1e-6
    for k in M.PARAM_NAMES:
        p = getattr(net, k)
        for idx in [tuple(0 for _ in p.shape), tuple(s - 1 for s in p.shape),
                    tuple(s // 2 for s in p.shape)]:
            old = p[idx]
            p[idx] = old + h
            lp, _ = net.loss_and_grads(Y, U)
            p[idx] = old - h
            lm, _ = net.loss_and_grads(Y, U)
            p[idx] = old
            np.testing.assert_allclose(g[k][idx], (lp - lm) / (2 * h), rtol=1e-6, atol=1e-10)


def test_first_adam_step_is_lr_times_sign():
    rng = np.random.default_rng(1)
    net = _tiny()
    before = net.params()
    before = {k: v.copy() for k, v in before.items()}
    _, g = net.loss_and_grads(rng.poisson(2.0, size=(4, 16)), rng.normal(size=(4, 3)))
    net.adam_step(g, lr=1e-3, eps=1e-12)
    for k in M.PARAM_NAMES:
        mask = np.abs(g[k]) > 1e-9
        np.testing.assert_allclose((before[k] - getattr(net, k))[mask], 1e-3 * np.sign(g[k][mask]),
                                   rtol=1e-6)


def test_training_learns_a_smooth_map():
    rng = np.random.default_rng(2)
    net = _tiny()
    Y = rng.poisson(3.0, size=(400, 16))
    U = np.log1p(Y[:, :3]) - 1.0
    losses = net.train(Y, U, epochs=40, batch=32, lr=3e-3)
    assert losses[-1] < 0.2 * losses[0]
