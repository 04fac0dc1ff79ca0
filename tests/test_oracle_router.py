"""Pins of the oracle parts behind the learned router: the weight-deviation
label, the linear component-wise flux, the stencil features and the MLP
gradient (against finite differences, not against its own formulas)."""
import numpy as np
import pytest

from oracle import mlp


def smooth_stencil(orc, amp, seed=0):
    rng = np.random.default_rng(seed)
    W = np.array([1.0, 0.3, 0.1, -0.2, 0.8, 0.5, -0.3, 0.9])
    ph = rng.uniform(0, 6, size=8)
    return np.array([orc.prim_to_cons(W + amp * np.sin(0.3 * j + ph)) for j in range(6)])


def test_linear_flux_equals_characteristic_flux_with_linear_weights(orc):
    # With linear weights (eps -> inf) and one LF speed for every field the
    # characteristic flux is R (linear scheme) L F = the component-wise linear
    # scheme, since R L = I: an identity between two independent code paths.
    for seed in range(10):
        Us = smooth_stencil(orc, 0.2, seed)
        Fc, _ = orc.interface_flux_ex(Us, eps=1e30, common_alpha=True)
        Fl = orc.linear_flux(Us)
        assert np.abs(Fc - Fl).max() < 1e-13 * (1 + np.abs(Fl).max())


def test_linear_flux_consistency_and_upwinding(orc):
    # uniform stencil -> physical flux; supersonic flow to the right -> the
    # F^- part vanishes only if alpha = |v| + c_f, which it is.
    Us = np.tile(orc.prim_to_cons(np.array([1.0, 0.3, 0.1, -0.2, 0.8, 0.5, -0.3, 0.9])), (6, 1))
    F = orc.flux(Us[0], 0)
    assert np.abs(orc.linear_flux(Us) - F).max() < 1e-14 * (1 + np.abs(F).max())


def test_weight_deviation_label(orc):
    # smooth small-amplitude data: weights within O(IS/eps) of linear; a
    # jump: some weight near 0 or 1, far from linear
    _, dev = orc.interface_flux_ex(smooth_stencil(orc, 1e-5))
    assert dev < 1e-4
    W1 = np.array([1.0, 0, 0, 0, 0.75, 1.0, 0, 1.0])
    W2 = np.array([0.125, 0, 0, 0, 0.75, -1.0, 0, 0.1])
    Us = np.array([orc.prim_to_cons(W1 if j < 3 else W2, 2.0) for j in range(6)])
    _, dev = orc.interface_flux_ex(Us, gamma=2.0)
    assert dev > 0.3
    # deviation does not change the flux itself
    F0 = orc.interface_flux(Us, gamma=2.0)
    F1, _ = orc.interface_flux_ex(Us, gamma=2.0)
    assert np.array_equal(F0, F1)


def test_features_invariances():
    rng = np.random.default_rng(1)
    s = rng.normal(size=(5, 6, 8))
    x = mlp.features(s)
    assert x.shape == (5, 48)
    assert np.abs(x).max() <= 1.0 + 1e-15
    # each variable attains |x| = 1 somewhere on the stencil
    assert np.allclose(np.abs(x.reshape(5, 8, 6)).max(-1), 1.0)
    # invariant under per-variable shifts and positive scalings, odd under sign flips
    a = rng.uniform(0.1, 10, size=8)
    b = rng.normal(size=8)
    assert np.allclose(mlp.features(s * a + b), x, atol=1e-12)
    assert np.allclose(mlp.features(-s), -x, atol=1e-12)
    # a constant variable gives zeros
    s2 = s.copy()
    s2[:, :, 3] = 7.0
    assert np.all(mlp.features(s2).reshape(5, 8, 6)[:, 3] == 0.0)


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    theta = mlp.init_params(3)
    X = rng.normal(size=(37, 48))
    t = (rng.uniform(size=37) < 0.4).astype(float)
    g = mlp.grad(theta, X, t)
    idx = rng.choice(mlp.NPARAM, size=60, replace=False)
    idx = np.concatenate([idx, [mlp.NPARAM - 1, 0, 48 * 32 + 5]])
    for i in idx:
        h = 1e-6
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (mlp.loss(tp, X, t) - mlp.loss(tm, X, t)) / (2 * h)
        assert abs(fd - g[i]) < 1e-6 * (1 + abs(fd)), (i, fd, g[i])


def test_mlp_pack_roundtrip_and_size():
    theta = mlp.init_params(0)
    assert theta.size == mlp.NPARAM == 2657
    assert np.array_equal(mlp.pack(*mlp.unpack(theta)), theta)
