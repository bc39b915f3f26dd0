"""FP64 reference of the per-edge proposal network and its training step.

TEST INFRASTRUCTURE ONLY (see oracle/oracle.py).

Network: 8 edge features -> 64 (ReLU) -> 64 (ReLU) -> 1 logit.  Trained on
(features, target proposal) pairs grouped by sampling step with the
listwise softmax cross-entropy
    loss = (1/G) sum_g  - sum_{i in g} y_i log softmax(logits_g)_i,
so d loss / d logit_i = (softmax_i - y_i) / G.  Parameters are packed as
W1[8][64], b1[64], W2[64][64], b2[64], w3[64], b3 (4801 values), the layout
the learned proposal of the oracle and of the library share by definition.
"""
from __future__ import annotations

import numpy as np

IN, H = 8, 64
NPARAM = IN * H + H + H * H + H + H + 1


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    o = 0
    W1 = theta[o:o + IN * H].reshape(IN, H); o += IN * H
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    w3 = theta[o:o + H]; o += H
    b3 = theta[o:o + 1]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, np.ravel(b3)]).astype(np.float64)


def init(seed: int = 0, scale: float = 1.0) -> np.ndarray:
    """Initial parameters from the seeded generator shared with the tests."""
    from paper_2608_15390_amd.inputs import network_params
    return network_params(seed, scale)


def forward(theta, X):
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    Z1 = X @ W1 + b1
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ W2 + b2
    H2 = np.maximum(Z2, 0.0)
    L = H2 @ w3 + b3[0]
    return L, (X, Z1, H1, Z2, H2)


def softmax_groups(L, offsets):
    S = np.empty_like(L)
    for g in range(len(offsets) - 1):
        a, b = offsets[g], offsets[g + 1]
        z = L[a:b] - L[a:b].max()
        e = np.exp(z)
        S[a:b] = e / e.sum()
    return S


def loss_and_grad(theta, X, y, offsets):
    """Listwise softmax cross-entropy over groups and its analytic gradient."""
    G = len(offsets) - 1
    L, (Xc, Z1, H1, Z2, H2) = forward(theta, X)
    S = softmax_groups(L, offsets)
    loss = -np.sum(y * np.log(np.maximum(S, 1e-300))) / G
    dL = (S - y) / G
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    dw3 = H2.T @ dL
    db3 = np.array([dL.sum()])
    dH2 = np.outer(dL, w3) * (Z2 > 0)
    dW2 = H1.T @ dH2
    db2 = dH2.sum(0)
    dH1 = (dH2 @ W2.T) * (Z1 > 0)
    dW1 = Xc.T @ dH1
    db1 = dH1.sum(0)
    return loss, pack(dW1, db1, dW2, db2, dw3, db3)


def adam(theta, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def quantize(theta):
    """Snap every parameter to the inference grid: multiples of 1/64 in
    [-127/64, 127/64]."""
    return np.clip(np.rint(np.asarray(theta, dtype=np.float64) * 64.0), -127, 127) / 64.0


def bf16(x):
    """Round to bfloat16 (round to nearest even) and back to float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
