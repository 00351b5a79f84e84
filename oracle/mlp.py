"""FP64 oracle for the warm-start MLP: forward, MSE loss, backprop, Adam.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The warm-start network is an ordinary MLP (Eq. 3 of the paper) with tanh
hidden layers and an identity output layer, trained to minimise the mean
squared error with Adam — the loss and optimizer the paper names for its
surrogate training (Section 4.2).  Definitions used here:

* rows of X (batch B) are inputs; Yhat = NN(X) row by row;
* loss = sum((Yhat - Y)^2) / (B * m);
* Adam (Kingma & Ba): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
  theta <- theta - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np


def _act(kind, z):
    if kind == "identity":
        return z, np.ones_like(z)
    if kind == "tanh":
        c = np.cosh(z)
        return np.tanh(z), 1.0 / (c * c)
    raise ValueError(kind)


def forward(Ws, bs, acts, X):
    """Row-batched forward pass; returns (list of (z_l, a_l), Yhat)."""
    A = np.asarray(X, dtype=np.float64)
    cache = []
    for W, b, kind in zip(Ws, bs, acts):
        Z = A @ W.T + b[None, :]
        A_next, _ = _act(kind, Z)
        cache.append((A, Z))
        A = A_next
    return cache, A


def loss(Ws, bs, acts, X, Y):
    _, Yhat = forward(Ws, bs, acts, X)
    return float(np.sum((Yhat - Y) ** 2) / Yhat.size)


def grads(Ws, bs, acts, X, Y):
    """(loss, [dL/dW_l], [dL/db_l]) by plain backpropagation."""
    cache, Yhat = forward(Ws, bs, acts, X)
    Y = np.asarray(Y, dtype=np.float64)
    dA = 2.0 * (Yhat - Y) / Yhat.size
    gW = [None] * len(Ws)
    gb = [None] * len(Ws)
    for l in range(len(Ws) - 1, -1, -1):
        A_in, Z = cache[l]
        _, d1 = _act(acts[l], Z)
        dZ = dA * d1
        gW[l] = dZ.T @ A_in
        gb[l] = dZ.sum(axis=0)
        dA = dZ @ Ws[l]
    return float(np.sum((Yhat - Y) ** 2) / Yhat.size), gW, gb


def adam_step(params, grads_, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place on lists of arrays; t is the 1-based step."""
    for p, g, mi, vi in zip(params, grads_, m, v):
        mi *= b1
        mi += (1.0 - b1) * g
        vi *= b2
        vi += (1.0 - b2) * g * g
        mhat = mi / (1.0 - b1 ** t)
        vhat = vi / (1.0 - b2 ** t)
        p -= lr * mhat / (np.sqrt(vhat) + eps)
