"""FP64 reference of the warm-start network (oracle; test infrastructure only).

Not part of the paper: a three-layer perceptron (input -> width -> width ->
K logits, ReLU between layers) whose masked softmax over the valid action
slots gives a behavioural prior per (infoset, hand).  The loss of a row is
weight * sum_a -target_a log softmax_a over valid slots (target < 0 marks an
invalid slot).  Forward and backward are written out plainly in numpy FP64;
finite differences pin the backward pass.
"""
from __future__ import annotations

import numpy as np


def forward(p, X):
    Z1 = X @ p["W1"].T + p["b1"]
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ p["W2"].T + p["b2"]
    H2 = np.maximum(Z2, 0.0)
    Z3 = H2 @ p["W3"].T + p["b3"]
    return Z3, (X, Z1, H1, Z2, H2)


def loss_and_grad(p, X, T, w):
    """Weighted masked cross-entropy (summed over rows) and its gradient."""
    Z3, (X, Z1, H1, Z2, H2) = forward(p, X)
    valid = T >= 0
    Zm = np.where(valid, Z3, -np.inf)
    mx = Zm.max(axis=1, keepdims=True)
    e = np.where(valid, np.exp(Zm - mx), 0.0)
    P = e / e.sum(axis=1, keepdims=True)
    logP = np.where(valid, Zm - mx - np.log(e.sum(axis=1, keepdims=True)), 0.0)
    Tv = np.where(valid, T, 0.0)
    loss = float((w * -(Tv * logP).sum(axis=1)).sum())
    dZ3 = np.where(valid, w[:, None] * (P - Tv), 0.0)
    g = {}
    g["W3"] = dZ3.T @ H2
    g["b3"] = dZ3.sum(axis=0)
    dZ2 = (dZ3 @ p["W3"]) * (Z2 > 0)
    g["W2"] = dZ2.T @ H1
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ p["W2"]) * (Z1 > 0)
    g["W1"] = dZ1.T @ X
    g["b1"] = dZ1.sum(axis=0)
    return loss, g, P


def init(d_in, width, k, seed=0):
    rng = np.random.default_rng(seed)

    def lin(o, i):
        a = np.sqrt(6.0 / i)
        return rng.uniform(-a, a, size=(o, i)), np.zeros(o)
    W1, b1 = lin(width, d_in)
    W2, b2 = lin(width, width)
    W3, b3 = lin(k, width)
    return {"W1": W1, "b1": b1, "W2": W2, "b2": b2, "W3": W3, "b3": b3 * 0.0}


def adam_step(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
    """One Adam step (Kingma and Ba, ICLR 2015: moving averages of the
    gradient and its square, each divided by its bias correction 1 - beta^t)
    on the gradient g + wd * w.  Returns the new (w, m, v); t counts from 1."""
    gt = g + wd * w
    m = b1 * m + (1.0 - b1) * gt
    v = b2 * v + (1.0 - b2) * gt * gt
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v
