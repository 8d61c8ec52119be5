"""Plain float64 CPU forward and backward of the warm-start network; test
infrastructure only (tests/ and the benchmark's CPU leg).

Network: dense layers h_{l+1} = tanh(h_l W_l + b_l) for the hidden layers and
a linear output layer, W_l of shape (in, out). Loss over a batch of M rows:
L = 1/(2M) sum (pred - target)^2.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np


def forward(params: List[Tuple[np.ndarray, np.ndarray]], X: np.ndarray):
    """Returns the list of layer outputs [X, h_1, ..., pred]."""
    hs = [np.asarray(X, dtype=np.float64)]
    for li, (W, b) in enumerate(params):
        z = hs[-1] @ W + b
        hs.append(np.tanh(z) if li < len(params) - 1 else z)
    return hs


def loss_and_grads(params, X, T):
    hs = forward(params, X)
    M = X.shape[0]
    d = hs[-1] - T
    loss = 0.5 * np.sum(d * d) / M
    grads = [None] * len(params)
    dz = d / M
    for li in range(len(params) - 1, -1, -1):
        W, b = params[li]
        grads[li] = (hs[li].T @ dz, dz.sum(axis=0))
        if li > 0:
            dh = dz @ W.T
            dz = dh * (1.0 - hs[li] ** 2)
    return loss, grads


def init_params(sizes, seed=0):
    """Glorot-uniform weights, zero biases (float64)."""
    rng = np.random.default_rng(seed)
    params = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / (a + b))
        params.append((rng.uniform(-lim, lim, (a, b)), np.zeros(b)))
    return params
