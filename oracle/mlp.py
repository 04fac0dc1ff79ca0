"""FP64 oracle of the learned troubled-interface router (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by the tests and the benchmark's checks, never
by the product path; shares no code with the HIP library.

The router is not part of the paper's method: an MLP 48 -> 32 -> 32 -> 1 with ReLU and a sigmoid output, trained with binary
cross-entropy on labels the full method produces:

  features: the six stencil cells i-2..i+3 of an interface, eight conserved
            variables each in the sweep frame (rho, m_n, m_t1, m_t2, B_n,
            B_t1, B_t2, E); six features per variable v, x[v*6 + j], each
            L(y) = 1 + log2m(y / S_v + 1e-8) log10(2) / 4 of
              j = 0     the largest first difference on the stencil,
              j = 1     the jump across the interface |q_3 - q_2|,
              j = 2..4  the largest second, third and fourth difference,
              j = 5     the fifth difference (absolute values throughout),
            with the stencil scales of oracle.flux_excess (a = max(|v_n| +
            c_f); S = max rho, max(|m|_1 + rho a), max |B|_1 + sqrt(max rho) a,
            max E for mass, momenta, fields, energy).  log2m is Mitchell's
            approximation of log2 (exponent plus mantissa fraction of the
            single-precision value), which the kernels evaluate with two
            instructions.  On smooth data the m-th difference falls like
            (kh)^m, so smoothness and amplitude are both differences of O(1)
            features, which survive the BF16 rounding of the inputs.
  label:    1 iff the flux excess (oracle.flux_excess: the characteristic
            WENO flux against the linear component-wise flux, relative to
            the same stencil scales) exceeds LABEL_THRESHOLD.

Parameter vector (2657 values): W1 (32x48, row-major [out][in]), b1 (32),
W2 (32x32), b2 (32), w3 (32), b3 (1).
"""
from __future__ import annotations

import numpy as np

NIN, NH = 48, 32
NPARAM = NH * NIN + NH + NH * NH + NH + NH + 1
LABEL_THRESHOLD = 1e-3


def fast_speed(U, gamma=5.0 / 3.0):
    """Fast magnetosonic speed along the first axis of conserved states
    (..., 8): c_f^2 = (a^2 + b^2 + sqrt((a^2 + b^2)^2 - 4 a^2 b_n^2)) / 2,
    a^2 = gamma p / rho, b^2 = |B|^2 / rho, b_n^2 = B_n^2 / rho."""
    U = np.asarray(U, dtype=np.float64)
    rho = U[..., 0]
    B2 = (U[..., 4:7] ** 2).sum(-1)
    p = (gamma - 1.0) * (U[..., 7] - 0.5 * (U[..., 1:4] ** 2).sum(-1) / rho - 0.5 * B2)
    a2 = gamma * p / rho
    b2 = B2 / rho
    bn2 = U[..., 4] ** 2 / rho
    return np.sqrt(0.5 * (a2 + b2 + np.sqrt((a2 + b2) ** 2 - 4.0 * a2 * bn2)))


def log2m(y):
    """Mitchell's log2: for y = 2^e (1 + f), 0 <= f < 1, returns e + f,
    taken from the IEEE single-precision bit pattern of y."""
    y32 = np.asarray(y, dtype=np.float32)
    return y32.view(np.int32).astype(np.float64) * 2.0 ** -23 - 127.0


def features(stencil, gamma=5.0 / 3.0):
    """stencil (..., 6, 8) sweep-frame conserved values -> (..., 48)."""
    s = np.asarray(stencil, dtype=np.float64)
    a = (np.abs(s[..., 1]) / s[..., 0] + fast_speed(s, gamma)).max(-1)[..., None]     # (..., 1)
    rho = s[..., 0]
    sr = rho.max(-1)[..., None]
    sm = (np.abs(s[..., 1:4]).sum(-1) + rho * a).max(-1)[..., None]
    sb = np.abs(s[..., 4:7]).sum(-1).max(-1)[..., None] + np.sqrt(sr) * a
    se = s[..., 7].max(-1)[..., None]
    S = np.concatenate([sr, sm, sm, sm, sb, sb, sb, se], -1)                         # (..., 8)
    y = [np.abs(np.diff(s, n=1, axis=-2)).max(-2), np.abs(s[..., 3, :] - s[..., 2, :])]
    y += [np.abs(np.diff(s, n=k, axis=-2)).max(-2) for k in (2, 3, 4, 5)]
    x = np.stack([1.0 + 0.25 * np.log10(2.0) * log2m(yk / S + 1e-8) for yk in y], -1)  # (..., 8, 6)
    return x.reshape(s.shape[:-2] + (NIN,))


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
