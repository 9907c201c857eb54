"""FP64 reference of the warm-start network (forward, MSE loss, gradients).

TEST INFRASTRUCTURE ONLY (see the package docstring).  The network is a
plain multilayer perceptron, widths w0 -> ... -> wL, ReLU after every layer
but the last, loss L = mean((Y - T)^2) over all entries.  Backpropagation is
written out layer by layer.

The optional argument q is applied to both operands of every matrix product
(identity by default).  With q = bf16_round it models a network whose
products take BF16 operands: the input, the weights, the hidden activations
and the back-propagated error each rounded (through FP32) to BF16, sums and
biases kept exact; the ReLU mask in the backward pass is the sign of the
rounded activation.
"""
from __future__ import annotations

import numpy as np


def _ident(a):
    return np.asarray(a, dtype=np.float64)


def forward(Ws, bs, X, q=None):
    """Returns the output and the list of layer inputs (activations, as
    they enter the products)."""
    q = q or _ident
    H = [q(X)]
    for l, (W, b) in enumerate(zip(Ws, bs)):
        Z = H[-1] @ q(W).T + np.asarray(b, np.float64)
        if l < len(Ws) - 1:
            H.append(q(np.maximum(Z, 0.0)))
        else:
            return Z, H
    raise ValueError("empty network")


def loss_and_grads(Ws, bs, X, T, q=None):
    q = q or _ident
    Y, H = forward(Ws, bs, X, q)
    T = np.asarray(T, np.float64)
    D = Y - T
    L = float(np.mean(D * D))
    G = 2.0 * D / D.size                       # dL/dY
    dWs, dbs = [None] * len(Ws), [None] * len(Ws)
    for l in range(len(Ws) - 1, -1, -1):
        dWs[l] = q(G).T @ H[l]
        dbs[l] = G.sum(axis=0)
        if l > 0:
            G = (q(G) @ q(Ws[l])) * (H[l] > 0)
    return L, dWs, dbs


def bf16_round(a):
    """Round FP32 values to BF16 (nearest, ties to even), returned as FP64."""
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
