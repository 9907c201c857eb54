"""FP64 reference of the warm-start network (forward, MSE loss, gradients).

TEST INFRASTRUCTURE ONLY (see the package docstring).  The network is a
plain multilayer perceptron, widths w0 -> ... -> wL, ReLU after every layer
but the last, loss L = mean((Y - T)^2) over all entries.  Backpropagation is
written out layer by layer.
"""
from __future__ import annotations

import numpy as np


def forward(Ws, bs, X):
    """Returns the output and the list of layer inputs (activations)."""
    H = [np.asarray(X, dtype=np.float64)]
    for l, (W, b) in enumerate(zip(Ws, bs)):
        Z = H[-1] @ np.asarray(W, np.float64).T + np.asarray(b, np.float64)
        if l < len(Ws) - 1:
            H.append(np.maximum(Z, 0.0))
        else:
            return Z, H
    raise ValueError("empty network")


def loss_and_grads(Ws, bs, X, T):
    Y, H = forward(Ws, bs, X)
    T = np.asarray(T, np.float64)
    D = Y - T
    L = float(np.mean(D * D))
    G = 2.0 * D / D.size                       # dL/dY
    dWs, dbs = [None] * len(Ws), [None] * len(Ws)
    for l in range(len(Ws) - 1, -1, -1):
        dWs[l] = G.T @ H[l]
        dbs[l] = G.sum(axis=0)
        if l > 0:
            G = (G @ np.asarray(Ws[l], np.float64)) * (H[l] > 0)
    return L, dWs, dbs


def bf16_round(a):
    """Round FP32 values to BF16 (nearest, ties to even), returned as FP64."""
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
