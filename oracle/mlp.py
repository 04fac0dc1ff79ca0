"""FP64 oracle of the learned troubled-interface router (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by the tests and the benchmark's checks, never
by the product path; shares no code with the HIP library.

The router is the learned part of this build (it is not in the paper): an
MLP 48 -> 32 -> 32 -> 1 with ReLU and a sigmoid output, trained with binary
cross-entropy on labels the full method produces:

  features: the six stencil cells i-2..i+3 of an interface, eight conserved
            variables each in the sweep frame (rho, m_n, m_t1, m_t2, B_n,
            B_t1, B_t2, E), each variable normalised over the stencil as
            (q - mean) / (max |q - mean| + 1e-30); ordered x[v*6 + j];
  label:    1 iff some weight of eq. (3) (any field, either side of eq. (1))
            deviates from the linear weights (0.1, 0.6, 0.3) by more than
            1e-2 (the oracle's interface_flux_ex gives the deviation).

Parameter vector (2657 values): W1 (32x48, row-major [out][in]), b1 (32),
W2 (32x32), b2 (32), w3 (32), b3 (1).
"""
from __future__ import annotations

import numpy as np

NIN, NH = 48, 32
NPARAM = NH * NIN + NH + NH * NH + NH + NH + 1
LABEL_THRESHOLD = 1e-2


def features(stencil):
    """stencil (..., 6, 8) sweep-frame conserved values -> (..., 48)."""
    s = np.asarray(stencil, dtype=np.float64)
    mean = s.mean(axis=-2, keepdims=True)
    dev = s - mean
    scale = np.abs(dev).max(axis=-2, keepdims=True) + 1e-30
    x = dev / scale
    return np.swapaxes(x, -1, -2).reshape(s.shape[:-2] + (NIN,))


def unpack(theta):
    t = np.asarray(theta, dtype=np.float64)
    o = 0
    W1 = t[o:o + NH * NIN].reshape(NH, NIN); o += NH * NIN
    b1 = t[o:o + NH]; o += NH
    W2 = t[o:o + NH * NH].reshape(NH, NH); o += NH * NH
    b2 = t[o:o + NH]; o += NH
    w3 = t[o:o + NH]; o += NH
    b3 = t[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [b3]])


def init_params(seed):
    """He-normal weights, zero biases."""
    g = np.random.Generator(np.random.PCG64(seed))
    W1 = g.standard_normal((NH, NIN)) * np.sqrt(2.0 / NIN)
    W2 = g.standard_normal((NH, NH)) * np.sqrt(2.0 / NH)
    w3 = g.standard_normal(NH) * np.sqrt(2.0 / NH)
    return pack(W1, np.zeros(NH), W2, np.zeros(NH), w3, 0.0)


def forward(theta, X):
    """X (B, 48) -> dict of activations and the logit (B,)."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    logit = h2 @ w3 + b3
    return {"z1": z1, "h1": h1, "z2": z2, "h2": h2, "logit": logit}


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def loss(theta, X, t):
    """Mean binary cross-entropy of sigmoid(logit) against labels t."""
    z = forward(theta, X)["logit"]
    return float(np.mean(np.logaddexp(0.0, z) - t * z))


def grad(theta, X, t):
    """Analytic gradient of loss() (chain rule through the two ReLU layers)."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    a = forward(theta, X)
    B = X.shape[0]
    g = (sigmoid(a["logit"]) - t) / B              # d loss / d logit
    dw3 = a["h2"].T @ g
    db3 = g.sum()
    d2 = np.outer(g, w3) * (a["z2"] > 0)           # (B, 32)
    dW2 = d2.T @ a["h1"]
    db2 = d2.sum(0)
    d1 = (d2 @ W2) * (a["z1"] > 0)
    dW1 = d1.T @ X
    db1 = d1.sum(0)
    return pack(dW1, db1, dW2, db2, dw3, db3)
