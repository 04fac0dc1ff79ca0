"""Pins of the oracle parts behind the learned router: the weight deviation,
the flux-excess label, the linear component-wise flux, the stencil features and the MLP
gradient (against finite differences, not against its own formulas)."""
import math

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


def test_linear_flux_central_plus_dissipation_form(orc):
    # The GPU evaluates the linear flux as (1,-8,37,37,-8,1)/60 F plus
    # alpha (1,-5,10,-10,5,-1)/60 U; with F+- = (F +- alpha U)/2 that is the
    # oracle's upwind pair (2,-13,47,27,-3)/60 on F+ and its mirror on F-.
    # Checked here against the oracle's own linear flux on smooth and on
    # discontinuous stencils, alpha = max(|v_n| + c_f) over the stencil.
    cen = np.array([1.0, -8.0, 37.0, 37.0, -8.0, 1.0]) / 60.0
    dis = np.array([1.0, -5.0, 10.0, -10.0, 5.0, -1.0]) / 60.0
    keep = [0, 1, 2, 3, 5, 6, 7]                      # every component but B_n
    rng = np.random.default_rng(11)
    for seed in range(12):
        if seed < 8:
            Us = smooth_stencil(orc, 0.2, seed)
        else:
            WL = np.concatenate([[rng.uniform(0.2, 2)], rng.normal(size=6), [rng.uniform(0.1, 2)]])
            WR = np.concatenate([[rng.uniform(0.2, 2)], rng.normal(size=6), [rng.uniform(0.1, 2)]])
            WR[4] = WL[4]
            Us = np.array([orc.prim_to_cons(WL if j < 3 else WR) for j in range(6)])
        F = np.array([orc.flux(U, 0) for U in Us])
        alpha = max(abs(U[1] / U[0]) + orc.wave_speeds(U, 0)[0] for U in Us)
        mine = cen @ F + alpha * (dis @ Us)
        ref = orc.linear_flux(Us)
        assert np.abs(mine[keep] - ref[keep]).max() < 1e-13 * (1 + np.abs(ref).max() + alpha * np.abs(Us).max())


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


def test_flux_excess_label(orc):
    # uniform stencil: both fluxes are the physical flux -> rounding only
    W0 = np.array([1.0, 0.5, 0.2, -0.1, 0.3, 0.2, 0.1, 1.0])
    assert orc.flux_excess(np.tile(orc.prim_to_cons(W0), (6, 1))) < 1e-14
    # smooth waves: the two fifth-order fluxes differ at O(h^5), so the
    # excess falls by ~2^5 per halving of the cell width
    worst = []
    for lam in (32, 64, 128):
        ex = []
        for ph in np.linspace(0, 2 * np.pi, 8, endpoint=False):
            Us = np.array([orc.prim_to_cons(W0 * (1 + 0.1 * np.sin(2 * np.pi * j / lam + ph + np.arange(8))))
                           for j in range(6)])
            ex.append(orc.flux_excess(Us))
        worst.append(max(ex))
    assert worst[0] < 1e-5
    assert worst[0] / worst[1] > 16 and worst[1] / worst[2] > 16, worst
    # tiny amplitude: linear weights and nearly equal speeds
    assert orc.flux_excess(smooth_stencil(orc, 1e-5)) < 1e-8
    # a Brio-Wu jump between cells 2 and 3: O(0.1)
    W1 = np.array([1.0, 0, 0, 0, 0.75, 1.0, 0, 1.0])
    W2 = np.array([0.125, 0, 0, 0, 0.75, -1.0, 0, 0.1])
    Us = np.array([orc.prim_to_cons(W1 if j < 3 else W2, 2.0) for j in range(6)])
    assert orc.flux_excess(Us, gamma=2.0) > 1e-2


def test_fast_speed_matches_c_oracle(orc):
    rng = np.random.default_rng(4)
    for _ in range(20):
        W = np.concatenate([[rng.uniform(0.1, 3)], rng.normal(size=3), rng.normal(size=3), [rng.uniform(0.05, 3)]])
        U = orc.prim_to_cons(W)
        assert abs(mlp.fast_speed(U) - orc.wave_speeds(U, 0)[0]) < 1e-13 * orc.wave_speeds(U, 0)[0]


def mitchell(z):
    # log2 z ~ (e - 1) + (2 f - 1) for z = f 2^e, f in [1/2, 1)
    f, e = math.frexp(z)
    return (e - 1) + (2 * f - 1)


def test_mitchell_log2():
    assert all(mlp.log2m(2.0 ** k) == k for k in range(-30, 30))
    z = np.exp(np.linspace(-20, 20, 5001))
    err = np.log2(z) - mlp.log2m(z)
    assert err.min() > -1e-6 and err.max() < 0.0861
    assert np.allclose(mlp.log2m(z), [mitchell(float(np.float32(v))) for v in z], atol=1e-12)


def test_features_definition(orc):
    W0 = np.array([1.0, 0.5, 0.2, -0.1, 0.3, 0.2, 0.1, 1.0])
    U0 = orc.prim_to_cons(W0)
    L = lambda y, S: 1 + 0.25 * math.log10(2.0) * mitchell(float(np.float32(y / S + 1e-8)))
    L0 = L(0.0, 1.0)
    # uniform stencil: every difference is 0 -> L(0)
    x = mlp.features(np.tile(U0, (6, 1))).reshape(8, 6)
    assert np.allclose(x, L0, atol=1e-15)
    # only rho alternates 1, 1.1, 1, ...: |differences| 0.1, 0.2, 0.4, 0.8,
    # 1.6, interface jump 0.1; mass scale max rho = 1.1
    st = np.tile(U0, (6, 1))
    st[:, 0] = [1.0, 1.1, 1.0, 1.1, 1.0, 1.1]
    x = mlp.features(st).reshape(8, 6)
    assert np.allclose(x[0], [L(0.1, 1.1), L(0.1, 1.1), L(0.2, 1.1), L(0.4, 1.1), L(0.8, 1.1), L(1.6, 1.1)],
                       atol=1e-12)
    assert np.allclose(x[1:], L0, atol=1e-15)
    # energy quadratic in the cell index: third and higher differences vanish
    st = np.tile(U0, (6, 1))
    st[:, 7] = U0[7] + 0.125 * np.arange(6) ** 2
    x = mlp.features(st).reshape(8, 6)[7]
    assert np.allclose(x[3:], L0, atol=1e-7) and x[2] > x[3] + 1
    # a resolved sine (kh = 2 pi / 64): the fifth difference sits ~(kh)^4,
    # i.e. ~4 decades (one feature unit), below the first
    lam = 64
    st = np.array([orc.prim_to_cons(W0 * (1 + 0.1 * np.sin(2 * np.pi * j / lam + np.arange(8)))) for j in range(6)])
    x = mlp.features(st).reshape(8, 6)
    assert np.all(x[:, 5] - x[:, 0] < -0.75)
    # random physical stencils: finite, at least -1
    rng = np.random.default_rng(1)
    for _ in range(10):
        st = np.array([orc.prim_to_cons(W0 * (1 + 0.3 * rng.normal(size=8)) * [1, 1, 1, 1, 1, 1, 1, 0] +
                                        [0, 0, 0, 0, 0, 0, 0, 1]) for _ in range(6)])
        x = mlp.features(st)
        assert np.all(np.isfinite(x)) and x.min() >= L0


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


def test_linear_rhs_converges_at_fifth_order(orc):
    # The all-linear scheme (the router's cheap flux everywhere) is a linear
    # fifth-order scheme: 1-D Alfven wave over one period, n = 16, 32, 64.
    from paper_1808_10633_amd import inputs as I
    import math
    errs = []
    for n in (16, 32, 64):
        u, speed = I.linear_wave_1d("alfven", n, amp=1e-5)
        g = orc.Grid(n, dx=1.0 / n)
        T = 1.0 / abs(speed)
        nst = int(math.ceil(T / (0.4 / n / 2.0)))
        dt = T / nst
        for _ in range(nst):
            k1 = orc.rhs_linear(g, u)
            k2 = orc.rhs_linear(g, u + 0.5 * dt * k1)
            k3 = orc.rhs_linear(g, u + 0.5 * dt * k2)
            k4 = orc.rhs_linear(g, u + dt * k3)
            u = u + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        ue, _ = I.linear_wave_1d("alfven", n, amp=1e-5, t=T)
        e = np.abs(g.interior(u) - g.interior(ue)).mean(axis=(1, 2, 3))
        errs.append(math.sqrt((e ** 2).sum()))
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert (order > 4.7).all(), (errs, order)
