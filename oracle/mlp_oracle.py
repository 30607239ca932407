"""FP64 CPU oracle of the learned warm-start encoder.

TEST INFRASTRUCTURE: only the tests, the smoke entry point and the benchmark's
CPU-baseline leg use it; it shares no code with the HIP kernels.

The encoder maps a row's counts to latent scores:
    x = log(1 + y) in R^m,
    h1 = gelu(W1 x + b1), h2 = gelu(W2 h1 + b2), out = W3 h2 + b3 in R^d,
with gelu(z) = z * Phi(z) = 0.5 z (1 + erf(z / sqrt 2)) (the exact GELU).
Training minimises the mean squared error
    L = 1 / (B d) * sum_{rows, k} (out - u)^2
over a minibatch of B rows, with Adam (Kingma and Ba 2014): for every
parameter, m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
theta <- theta - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
- lr wd theta (decoupled weight decay when wd > 0), t counting updates.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.special import erf


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    """d gelu / dz = Phi(z) + z phi(z)."""
    phi = np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * phi


PARAM_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


@dataclass
class MLP:
    W1: np.ndarray   # H x m
    b1: np.ndarray   # H
    W2: np.ndarray   # H x H
    b2: np.ndarray   # H
    W3: np.ndarray   # d x H
    b3: np.ndarray   # d
    adam_m: dict = field(default_factory=dict)
    adam_v: dict = field(default_factory=dict)
    t: int = 0

    def params(self):
        return {k: getattr(self, k) for k in PARAM_NAMES}

    def copy(self):
        return MLP(*(np.array(getattr(self, k), dtype=np.float64) for k in PARAM_NAMES))

    def forward(self, Y):
        x = np.log1p(np.asarray(Y, np.float64))
        z1 = x @ self.W1.T + self.b1
        h1 = gelu(z1)
        z2 = h1 @ self.W2.T + self.b2
        h2 = gelu(z2)
        out = h2 @ self.W3.T + self.b3
        return out, (x, z1, h1, z2, h2)

    def loss_and_grads(self, Y, U):
        out, (x, z1, h1, z2, h2) = self.forward(Y)
        B, d = out.shape
        r = out - U
        loss = float(np.sum(r * r) / (B * d))
        dout = 2.0 * r / (B * d)
        g = {}
        g["W3"] = dout.T @ h2
        g["b3"] = dout.sum(axis=0)
        dz2 = (dout @ self.W3) * gelu_grad(z2)
        g["W2"] = dz2.T @ h1
        g["b2"] = dz2.sum(axis=0)
        dz1 = (dz2 @ self.W2) * gelu_grad(z1)
        g["W1"] = dz1.T @ x
        g["b1"] = dz1.sum(axis=0)
        return loss, g

    def adam_step(self, grads, lr, beta1=0.9, beta2=0.999, eps=1e-8, wd=0.0):
        self.t += 1
        for k in PARAM_NAMES:
            p = getattr(self, k)
            m = self.adam_m.get(k, np.zeros_like(p))
            v = self.adam_v.get(k, np.zeros_like(p))
            gk = grads[k]
            m = beta1 * m + (1 - beta1) * gk
            v = beta2 * v + (1 - beta2) * gk * gk
            mh = m / (1 - beta1 ** self.t)
            vh = v / (1 - beta2 ** self.t)
            p = p - lr * mh / (np.sqrt(vh) + eps) - lr * wd * p
            setattr(self, k, p)
            self.adam_m[k], self.adam_v[k] = m, v

    def train(self, Y, U, epochs, batch, lr, **adam):
        """Minibatches of `batch` consecutive rows in the given order, every epoch."""
        losses = []
        n = Y.shape[0]
        for _ in range(epochs):
            tot = 0.0
            for b0 in range(0, n, batch):
                loss, g = self.loss_and_grads(Y[b0:b0 + batch], U[b0:b0 + batch])
                self.adam_step(g, lr, **adam)
                tot += loss * min(batch, n - b0)
            losses.append(tot / n)
        return losses
