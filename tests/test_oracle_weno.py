"""Pins of the oracle's scalar WENO5 (arXiv:1808.10633 Sec. 2.1, eqs. 1-7)
against facts the paper and the mathematics fix, not against its own code."""
import numpy as np
import pytest

D_LINEAR = np.array([0.1, 0.6, 0.3])   # alpha numerators 1:6:3 of eq. (4)


def test_linear_data_gives_linear_weights(orc):
    # a=b=c=d makes IS_0 = IS_1 = IS_2 = 12 a^2 (eqs. 5-7), so eq. (3) gives
    # the linear weights for any epsilon.
    rng = np.random.default_rng(1)
    for a in np.concatenate([rng.normal(size=20), [0.0, 1e-8, 1e4]]):
        w, s = orc.weno_weights(a, a, a, a)
        assert np.allclose(s, 12 * a * a, rtol=1e-15, atol=0)
        assert np.abs(w - D_LINEAR).max() < 4e-16


def test_weights_tend_to_linear_for_small_amplitude(orc):
    rng = np.random.default_rng(2)
    x = rng.normal(size=4)
    prev = None
    for amp in (1e-4, 1e-5, 1e-6):
        w, s = orc.weno_weights(*(amp * x))
        dev = np.abs(w - D_LINEAR).max()
        # deviation is O(IS/eps) with IS ~ amp^2
        assert dev < 50 * amp * amp / 1e-6
        if prev is not None:
            assert dev < prev / 50
        prev = dev


def test_phi_with_linear_weights_closed_form(orc):
    # With omega = (0.1, 0.6, 0.3), eq. (2) reduces to (a - 3b + 3c - d)/30.
    rng = np.random.default_rng(3)
    for _ in range(50):
        a, b, c, d = rng.normal(size=4)
        got = orc.weno_phi(a, b, c, d, eps=1e30)
        assert abs(got - (a - 3 * b + 3 * c - d) / 30) < 1e-15


def test_phi_is_odd(orc):
    rng = np.random.default_rng(4)
    for _ in range(50):
        a, b, c, d = rng.normal(size=4) * 10 ** rng.uniform(-4, 2)
        assert orc.weno_phi(-a, -b, -c, -d) == -orc.weno_phi(a, b, c, d)


def test_eno_weights_at_a_step(orc):
    # Jump between c and d-stencils: IS = (0, 16, 40); the two stencils that
    # cross the jump get weights ~2e-14 and ~2e-15.
    w, s = orc.weno_weights(0.0, 0.0, 1.0, 0.0)
    assert np.allclose(s, [0.0, 16.0, 40.0])
    assert 1e-14 < w[1] < 5e-14
    assert 1e-15 < w[2] < 5e-15
    assert abs(w[0] - 1.0) < 1e-13


def test_upwind_flux_closed_form(orc):
    # Pure right-moving data (u = f, alpha = 1 -> F^- = 0) with linear weights:
    # eq. (1) becomes the fifth-order upwind flux
    # (2 f_{i-2} - 13 f_{i-1} + 47 f_i + 27 f_{i+1} - 3 f_{i+2}) / 60.
    rng = np.random.default_rng(5)
    for _ in range(50):
        f = rng.normal(size=6)
        got = orc.weno_field_flux(f, f, 1.0, eps=1e30)
        want = (2 * f[0] - 13 * f[1] + 47 * f[2] + 27 * f[3] - 3 * f[4]) / 60
        assert abs(got - want) < 2e-15 * (1 + np.abs(f).max())
        # and the mirror image for left-moving data (u = -f)
        got = orc.weno_field_flux(f, -f, 1.0, eps=1e30)
        want = (-3 * f[1] + 27 * f[2] + 47 * f[3] - 13 * f[4] + 2 * f[5]) / 60
        assert abs(got - want) < 2e-15 * (1 + np.abs(f).max())


def test_mirror_symmetry(orc):
    # Reversing the stencil and the sign of f maps F^+ onto F^- and back, so
    # eq. (1) must return the negated flux (up to rounding order).
    rng = np.random.default_rng(6)
    for _ in range(100):
        f = rng.normal(size=6) * 10 ** rng.uniform(-3, 1)
        u = rng.normal(size=6)
        al = abs(rng.normal()) + 0.1
        a = orc.weno_field_flux(f, u, al)
        b = orc.weno_field_flux(-f[::-1].copy(), u[::-1].copy(), al)
        # equal up to the summation order of the central term
        assert abs(a + b) <= 4e-16 * (np.abs(f).max() + al * np.abs(u).max())


@pytest.mark.parametrize("degree", [0, 1, 2, 3, 4, 5])
def test_flux_difference_exact_for_polynomials(orc, degree):
    # With linear weights the flux difference is a six-point fifth-order
    # derivative, exact for polynomials of degree <= 5, for any split speed.
    rng = np.random.default_rng(10 + degree)
    cf = rng.normal(size=degree + 1)
    cu = rng.normal(size=degree + 1)
    h = 0.1
    x = (np.arange(-4, 4) + 0.3) * h    # cells i-4 .. i+3 around cell i (index 4)
    f = np.polyval(cf, x)
    u = np.polyval(cu, x)
    alpha = 1.7
    Fr = orc.weno_field_flux(f[2:8], u[2:8], alpha, eps=1e30)   # i+1/2: cells i-2..i+3
    Fl = orc.weno_field_flux(f[1:7], u[1:7], alpha, eps=1e30)   # i-1/2: cells i-3..i+2
    deriv = np.polyval(np.polyder(cf), x[4]) if degree > 0 else 0.0
    assert abs((Fr - Fl) / h - deriv) < 1e-11 * (1 + np.abs(cf).sum())


def test_interpolation_order_on_smooth_data(orc):
    # With the paper's epsilon, smooth data away from extrema converges at
    # fifth order (Sec. 2.1, eq. 1).
    errs = []
    for n in (20, 40, 80):
        h = 1.0 / n
        x = 0.3 + (np.arange(-4, 4)) * h
        f = np.exp(x)     # monotone, no critical points
        Fr = orc.weno_field_flux(f[2:8], f[2:8], 1.0)
        Fl = orc.weno_field_flux(f[1:7], f[1:7], 1.0)
        errs.append(abs((Fr - Fl) / h - np.exp(x[4])))
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert (order > 4.5).all(), order
