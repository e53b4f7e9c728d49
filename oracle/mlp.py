"""Float64 oracle of the cost-model MLP (test infrastructure only).

Network: x (B x 12) -> h1 = relu(x W1^T + b1) (64) -> h2 = relu(h1 W2^T + b2)
(64) -> y = h2 W3^T + b3 (2).  Weights W_l are (out x in), row-major.
Loss: L = 1/(2B) sum_{b,k} w_bk (y_bk - t_bk)^2 (w = 1 unless given; a zero
weight masks a missing target).  relu'(0) is taken as 0.
Backward: the chain rule written out layer by layer.
Optimiser: Adam (Kingma and Ba, 2015) with bias correction:
  m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;
  p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np


def forward(ws, bs, x):
    acts = [x]
    h = x
    for li, (w, b) in enumerate(zip(ws, bs)):
        z = h @ w.T + b
        h = np.maximum(z, 0.0) if li < len(ws) - 1 else z
        acts.append(h)
    return acts


def loss(y, t, w=None):
    w = 1.0 if w is None else w
    return 0.5 * float(np.sum(w * (y - t) ** 2)) / y.shape[0]


def backward(ws, bs, acts, t, w=None):
    """Gradients (dW_l, db_l) of the loss for every layer, float64."""
    B = t.shape[0]
    w = 1.0 if w is None else w
    g = w * (acts[-1] - t) / B  # dL/dy
    dws, dbs = [None] * len(ws), [None] * len(ws)
    for li in range(len(ws) - 1, -1, -1):
        h_in = acts[li]
        dws[li] = g.T @ h_in
        dbs[li] = g.sum(axis=0)
        if li > 0:
            g = (g @ ws[li]) * (acts[li] > 0.0)
    return dws, dbs


def adam_step(params, grads, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update, in place on params, m, v (lists of arrays)."""
    for p, g, mm, vv in zip(params, grads, m, v):
        mm *= b1
        mm += (1.0 - b1) * g
        vv *= b2
        vv += (1.0 - b2) * g * g
        mhat = mm / (1.0 - b1 ** t)
        vhat = vv / (1.0 - b2 ** t)
        p -= lr * mhat / (np.sqrt(vhat) + eps)
