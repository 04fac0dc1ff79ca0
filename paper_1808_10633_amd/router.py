"""Training and calibration of the learned troubled-interface router.

Every numerical step runs in the HIP library: interface sampling (features
and weight-deviation labels computed by the full characteristic WENO
kernel), the MLP forward/backward passes (BF16 MFMA, FP32 accumulation) and
the Adam update.  This module only draws random interface positions,
shuffles minibatches and keeps the loop.

Label of an interface ("troubled"): its flux excess (how far the
characteristic WENO flux of arXiv:1808.10633 Sec. 2.1 departs from the linear
component-wise flux, relative to the stencil's flux scale; the library
computes it while sampling) exceeds LABEL_THRESHOLD.  On smooth data the two
fifth-order fluxes differ at O(h^5), at a discontinuity at O(0.1).  The
deviation of the nonlinear weights from the linear ones is returned too; it
is not used as the label because the weights of eq. (3) depart from linear
by O((kh)^2) on smooth data and by O(1) near extrema of any characteristic
field, so a deviation threshold marks nearly every interface of a turbulent
box as troubled.
"""
from __future__ import annotations

import math

import numpy as np

from . import wombat

LABEL_THRESHOLD = 1e-3
NIN, NH = 48, 32


def init_params(seed, device="cuda"):
    """He-normal weights, zero biases, packed as the library expects."""
    import torch
    g = np.random.Generator(np.random.PCG64(seed))
    parts = [g.standard_normal(NH * NIN) * math.sqrt(2.0 / NIN), np.zeros(NH),
             g.standard_normal(NH * NH) * math.sqrt(2.0 / NH), np.zeros(NH),
             g.standard_normal(NH) * math.sqrt(2.0 / NH), np.zeros(1)]
    return torch.tensor(np.concatenate(parts), dtype=torch.float32, device=device)


def random_interfaces(shape, n, seed, device="cuda"):
    """n random interfaces (dir, i, j, k) of an (nx, ny, nz) box: the
    coordinate along dir is a face index 0..n_dir, the others interior."""
    import torch
    nx, ny, nz = shape
    g = np.random.Generator(np.random.PCG64(seed))
    d = g.integers(0, 3, size=n)
    lim = np.array([nx, ny, nz])
    pos = np.stack([g.integers(0, lim[a] + (d == a).astype(int)) for a in range(3)], 1)
    where = np.concatenate([d[:, None], pos], 1).astype(np.int32)
    return torch.from_numpy(where).to(device)


def sample(ctx, u, n, seed, threshold=LABEL_THRESHOLD):
    """(features (n, 48), weight deviation (n,), flux excess (n,), labels
    (n,)) at n random interfaces."""
    shape = (ctx.cfg.nx, ctx.cfg.ny, ctx.cfg.nz)
    X, dev, ex = ctx.router_sample(u, random_interfaces(shape, n, seed, u.device))
    return X, dev, ex, (ex > threshold).float()


def train(X, t, steps=2000, batch=4096, lr=2e-3, seed=0, pos_weight=None, log_every=0):
    """Adam on the mean BCE; returns (theta, list of (step, loss))."""
    import torch
    n = X.shape[0]
    theta = init_params(seed, X.device)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    work = torch.empty(int(wombat.lib().wombat_mlp_grad_workspace(batch)), dtype=torch.float32,
                       device=X.device)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    perm = torch.randperm(n, generator=gen).to(X.device)
    pos = 0
    for step in range(1, steps + 1):
        if pos + batch > n:
            perm = torch.randperm(n, generator=gen).to(X.device)
            pos = 0
        idx = perm[pos:pos + batch]
        pos += batch
        xb = X[idx].contiguous()
        tb = t[idx].contiguous()
        g, loss = wombat.mlp_grad(theta, xb, tb, work)
        wombat.mlp_adam(theta, m, v, g, step, lr=lr)
        if log_every and (step % log_every == 0 or step == 1):
            hist.append((step, float(loss)))
    return theta, hist


def evaluate(theta, X, t, threshold=0.5, excess=None):
    """Classifier statistics at a probability threshold; with the flux
    excess of the samples, also the largest and 99.9th-percentile excess
    among the interfaces it would route to the linear flux."""
    import torch
    z = wombat.mlp_forward(theta, X)
    pred = (z > math.log(threshold / (1.0 - threshold))).float()
    tr = t > 0.5
    n_tr = int(tr.sum())
    false_smooth = int(((pred < 0.5) & tr).sum())
    out = {"accuracy": float((pred == t).float().mean()),
           "troubled_fraction": float(t.mean()),
           "predicted_troubled_fraction": float(pred.mean()),
           "false_smooth_rate": false_smooth / max(n_tr, 1)}
    if excess is not None:
        es = excess[pred < 0.5].float()
        if es.numel():
            out["routed_smooth_excess_max"] = float(es.max())
            out["routed_smooth_excess_p999"] = float(torch.quantile(es[:1 << 24], 0.999))
    return out


def choose_threshold(theta, X, t, max_false_smooth=0.10):
    """Largest threshold whose false-smooth rate (troubled interfaces sent
    to the linear flux) stays at or below max_false_smooth."""
    z = wombat.mlp_forward(theta, X).double().cpu().numpy()
    tr = t.cpu().numpy() > 0.5
    zt = np.sort(z[tr])
    if zt.size == 0:
        return 0.5
    k = int(math.floor(max_false_smooth * zt.size))
    zthr = zt[k] - 1e-6
    p = 1.0 / (1.0 + math.exp(-zthr))
    return float(min(max(p, 1e-6), 1 - 1e-6))
