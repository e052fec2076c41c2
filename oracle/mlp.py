"""Two-layer tanh network, FP64 forward and backward (oracle; test infrastructure only).

Not in the paper: an element-local learned preconditioner added on top of the
method. The network is y = W2 tanh(W1 x + b1) + b2 acting on a batch of rows
x; the loss is the mean squared error over every output entry of the batch,
L = sum (y - t)^2 / (batch * out). The gradients below are the chain rule
written out; the tests pin them with central finite differences. Adam is the
published update of Kingma and Ba (2015), with bias correction.
"""
from __future__ import annotations

import numpy as np


def init_params(n_in: int, n_hidden: int, n_out: int, seed: int) -> dict:
    rng = np.random.default_rng(seed)
    return dict(
        W1=rng.uniform(-1, 1, (n_hidden, n_in)) / np.sqrt(n_in),
        b1=np.zeros(n_hidden),
        W2=rng.uniform(-1, 1, (n_out, n_hidden)) / np.sqrt(n_hidden),
        b2=np.zeros(n_out),
    )


def forward(params: dict, X: np.ndarray):
    Z = X @ params["W1"].T + params["b1"]
    H = np.tanh(Z)
    Y = H @ params["W2"].T + params["b2"]
    return Y, H


def loss(params: dict, X: np.ndarray, T: np.ndarray) -> float:
    Y, _ = forward(params, X)
    return float(np.sum((Y - T) ** 2) / Y.size)


def loss_and_grads(params: dict, X: np.ndarray, T: np.ndarray):
    Y, H = forward(params, X)
    L = float(np.sum((Y - T) ** 2) / Y.size)
    dY = 2.0 * (Y - T) / Y.size
    gW2 = dY.T @ H
    gb2 = dY.sum(axis=0)
    dH = dY @ params["W2"]
    dZ = dH * (1.0 - H * H)
    gW1 = dZ.T @ X
    gb1 = dZ.sum(axis=0)
    return L, dict(W1=gW1, b1=gb1, W2=gW2, b2=gb2)


def adam_step(params: dict, grads: dict, state: dict, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place; ``state`` holds m, v and the step count t."""
    t = state.get("t", 0) + 1
    state["t"] = t
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[...] = beta1 * m + (1 - beta1) * grads[k]
        v[...] = beta2 * v + (1 - beta2) * grads[k] ** 2
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        params[k] -= lr * mh / (np.sqrt(vh) + eps)
    return params
