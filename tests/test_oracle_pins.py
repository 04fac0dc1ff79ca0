"""Pins of two oracle parts that the other tests only compare with themselves.

orc_sums (the FP64 diagnostics every conservation test uses): against an
exact interior sum written independently here (Python's math.fsum, correctly
rounded), on states whose ghost zones hold large values and whose variables
have distinct magnitudes, so that summing a ghost cell, a wrong stride or a
wrong variable offset fails; and on 1-D/2-D boxes (inactive axes have no
ghosts).  Conservation by the flux form (Sec. 2.1) is checked through these
sums, so they must measure the interior and nothing else.

mlp.loss (the training objective of the learned router): against closed
forms of the mean binary cross-entropy of a sigmoid output, which the
finite-difference gradient test cannot distinguish from a sign or mean/sum
slip: zero parameters give log 2 for either label; a constant logit z gives
log(1 + e^-z) for label 1 and log(1 + e^z) for label 0; a batch of samples
gives the mean of the per-sample values; a confident correct prediction has a
loss near e^-|z|.
"""
import math

import numpy as np
import pytest

from oracle import mlp


def _padded(orc, nx, ny, nz, seed):
    g = orc.Grid(nx, ny, nz, 1.0 / nx, 1.0 / max(ny, 1), 1.0 / max(nz, 1))
    rng = np.random.default_rng(seed)
    u = np.empty(g.shape)
    for v in range(8):
        # distinct magnitude and sign pattern per variable
        u[v] = (v + 1) * 10.0 ** (v - 3) * (1.0 + rng.uniform(-0.5, 0.5, size=g.shape[1:]))
    # ghosts: huge values (a ghost cell in the sum is visible at once)
    gx, gy, gz = g.ghosts
    mask = np.ones(g.shape[1:], dtype=bool)
    mask[gz:gz + nz, gy:gy + ny, gx:gx + nx] = False
    u[:, mask] = 1e12 * (1 + np.arange(8))[:, None]
    return g, u


@pytest.mark.parametrize("dims", [(7, 6, 5), (9, 1, 1), (5, 8, 1), (1, 4, 6), (12, 12, 12)])
def test_sums_equal_exact_interior_sums(orc, dims):
    g, u = _padded(orc, *dims, seed=sum(dims))
    got = orc.sums(g, u)
    inner = g.interior(u)
    for v in range(8):
        ref = math.fsum(inner[v].ravel().tolist())
        scale = math.fsum(np.abs(inner[v]).ravel().tolist())
        assert abs(got[v] - ref) <= 4e-16 * scale, (dims, v, got[v], ref)


def test_sums_see_each_interior_cell_once(orc):
    # one interior cell raised by 1 changes exactly its variable's sum by 1
    g, u = _padded(orc, 6, 5, 4, seed=3)
    base = orc.sums(g, u)
    gx, gy, gz = g.ghosts
    for v, (i, j, k) in ((0, (0, 0, 0)), (3, (5, 4, 3)), (7, (2, 1, 3)), (5, (5, 0, 0))):
        w = u.copy()
        w[v, gz + k, gy + j, gx + i] += 1.0
        d = orc.sums(g, w) - base
        want = np.zeros(8)
        want[v] = 1.0
        assert np.allclose(d, want, rtol=0, atol=1e-9 * (1 + np.abs(base).max())), (v, d)


def test_sums_ignore_ghost_values(orc):
    g, u = _padded(orc, 6, 5, 4, seed=4)
    base = orc.sums(g, u)
    w = u.copy()
    gx, gy, gz = g.ghosts
    w[:, :gz] = -7.0
    w[:, :, :, -gx:] = 3.0e9
    assert np.array_equal(orc.sums(g, w), base)


def _theta_with_logit(z):
    """All weights zero, output bias z: every sample's logit is z."""
    th = np.zeros(mlp.NPARAM)
    th[-1] = z
    return th


def test_loss_zero_parameters_is_log2():
    X = np.random.default_rng(0).uniform(-1, 1, size=(17, mlp.NIN))
    for t in (np.zeros(17), np.ones(17), (np.arange(17) % 2).astype(float)):
        assert abs(mlp.loss(np.zeros(mlp.NPARAM), X, t) - math.log(2.0)) < 1e-15


@pytest.mark.parametrize("z", [-30.0, -3.0, -0.25, 0.0, 0.7, 4.0, 40.0])
def test_loss_closed_form_single_logit(z):
    X = np.zeros((1, mlp.NIN))
    th = _theta_with_logit(z)
    # label 1: -log(sigmoid(z)); label 0: -log(1 - sigmoid(z))
    pos = math.log1p(math.exp(-z)) if z > -30 else -z + math.log1p(math.exp(z))
    neg = math.log1p(math.exp(z)) if z < 30 else z + math.log1p(math.exp(-z))
    assert abs(mlp.loss(th, X, np.array([1.0])) - pos) <= 1e-13 * max(1.0, pos)
    assert abs(mlp.loss(th, X, np.array([0.0])) - neg) <= 1e-13 * max(1.0, neg)


def test_loss_is_the_mean_over_samples():
    # per-sample logits differ through the first-layer weights: logit = relu
    # chain of x_0; build it by hand with one hidden path of gain 1
    th = np.zeros(mlp.NPARAM)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(th)
    W1 = W1.copy(); W2 = W2.copy(); w3 = w3.copy()
    W1[0, 0] = 1.0          # h1_0 = relu(x_0)
    W2[0, 0] = 1.0          # h2_0 = relu(h1_0)
    w3[0] = 1.0             # logit = h2_0 + b3
    th = mlp.pack(W1, b1, W2, b2, w3, -1.0)
    xs = np.array([0.0, 0.5, 2.0, 5.0])
    X = np.zeros((4, mlp.NIN))
    X[:, 0] = xs
    t = np.array([1.0, 0.0, 1.0, 0.0])
    z = xs - 1.0
    per = [math.log1p(math.exp(-zz)) if tt == 1 else math.log1p(math.exp(zz)) for zz, tt in zip(z, t)]
    assert abs(mlp.loss(th, X, t) - sum(per) / 4) < 1e-15
    # duplicating the batch leaves the mean unchanged (a sum would double)
    assert abs(mlp.loss(th, np.vstack([X, X]), np.concatenate([t, t])) - sum(per) / 4) < 1e-15


def test_loss_confident_prediction():
    X = np.zeros((1, mlp.NIN))
    z = 25.0
    l = mlp.loss(_theta_with_logit(z), X, np.array([1.0]))
    assert 0 < l and abs(l - math.exp(-z)) < 1e-3 * math.exp(-z)
    # the wrong label costs about |z|
    assert abs(mlp.loss(_theta_with_logit(z), X, np.array([0.0])) - z) < 1e-9
