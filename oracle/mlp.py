"""FP64 reference of the learned candidate-proposal scorer -- test infrastructure only.

This form is not in the paper; it extends the method's candidate selection
(the extremes of Alg. 1 / Alg. 2) with points a small network scores as
likely Hausdorff witnesses.  The definitions below are this library's own:

* features of a point x of one set, with c the centroid of the OTHER set:
  ``f = [x, x - c]`` (2D values);
* ``z1 = W1 f + b1`` (256), ``h1 = gelu(z1)``; ``z2 = W2 h1 + b2`` (128),
  ``h2 = gelu(z2)``; score ``s = w3 . h2 + b3``; gelu is the exact
  ``0.5 z (1 + erf(z / sqrt 2))``;
* loss: mean over the batch of the binary cross-entropy with logits, the
  positive term weighted by ``pos_weight``:
  ``l = pos_weight * y * softplus(-s) + (1 - y) * softplus(s)``;
* AdamW: ``m = b1 m + (1-b1) g``, ``v = b2 v + (1-b2) g^2``,
  ``p -= lr * (m / (1-b1^t) / (sqrt(v / (1-b2^t)) + eps) + wd * p)``.

Flat parameter layout (both sides use it; nothing is shared but the
convention): ``[W1 (256 x 2D, row-major), b1 (256), W2 (128 x 256), b2
(128), w3 (128), b3 (1)]``.

Pins: central finite differences of the loss (tests/test_oracle_pins.py),
and a one-unit hand example.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

H1 = 256
H2 = 128

__all__ = ["H1", "H2", "param_count", "unpack", "features", "forward", "loss_grad", "adamw"]


def param_count(D: int) -> int:
    return H1 * 2 * D + H1 + H2 * H1 + H2 + H2 + 1


def unpack(p, D: int):
    """Views (W1, b1, W2, b2, w3, b3) into a flat parameter vector."""
    p = np.asarray(p)
    o = 0
    W1 = p[o:o + H1 * 2 * D].reshape(H1, 2 * D); o += H1 * 2 * D
    b1 = p[o:o + H1]; o += H1
    W2 = p[o:o + H2 * H1].reshape(H2, H1); o += H2 * H1
    b2 = p[o:o + H2]; o += H2
    w3 = p[o:o + H2]; o += H2
    b3 = p[o:o + 1]; o += 1
    assert o == p.size
    return W1, b1, W2, b2, w3, b3


def features(X, c_other):
    """[x, x - c] for every row x (float64)."""
    X = np.asarray(X, dtype=np.float64)
    c = np.asarray(c_other, dtype=np.float64)
    return np.hstack([X, X - c[None, :]])


def _gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def _gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(p, F, D: int):
    """Scores s (N,) and the intermediates (z1, h1, z2, h2)."""
    W1, b1, W2, b2, w3, b3 = unpack(np.asarray(p, dtype=np.float64), D)
    F = np.asarray(F, dtype=np.float64)
    z1 = F @ W1.T + b1
    h1 = _gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = _gelu(z2)
    s = h2 @ w3 + b3[0]
    return s, (z1, h1, z2, h2)


def _softplus(x):
    return np.logaddexp(0.0, x)


def loss_grad(p, F, y, D: int, pos_weight: float = 1.0):
    """Mean weighted BCE-with-logits and its gradient (flat, FP64)."""
    p = np.asarray(p, dtype=np.float64)
    W1, b1, W2, b2, w3, b3 = unpack(p, D)
    F = np.asarray(F, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    N = F.shape[0]
    s, (z1, h1, z2, h2) = forward(p, F, D)
    loss = float(np.mean(pos_weight * y * _softplus(-s) + (1.0 - y) * _softplus(s)))
    sig = 0.5 * (1.0 + np.tanh(0.5 * s))          # logistic sigmoid, stable
    ds = (pos_weight * y * (sig - 1.0) + (1.0 - y) * sig) / N
    gw3 = h2.T @ ds
    gb3 = np.array([ds.sum()])
    dz2 = np.outer(ds, w3) * _gelu_grad(z2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * _gelu_grad(z1)
    gW1 = dz1.T @ F
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gw3, gb3])
    return loss, g


def adamw(p, g, m, v, t: int, lr: float, wd: float = 0.01, b1: float = 0.9, b2: float = 0.999,
          eps: float = 1e-8):
    """One AdamW step (decoupled weight decay); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    p = p - lr * (mh / (np.sqrt(vh) + eps) + wd * p)
    return p, m, v
