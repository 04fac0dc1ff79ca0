"""Pins of the oracle's global Lax-Friedrichs speeds, the ablation of the
per-stencil speed (the reading of eq. (1)'s "simple Lax-Friedrichs
splitting" in arXiv:1808.10633 Sec. 2.1): facts of the splitting, not of the
oracle's code.

* Two-state data (a Riemann problem at t = 0): every stencil is uniform, where
  the flux does not depend on alpha, or holds both states, where its largest
  speed is the global one; the two right-hand sides are identical.
* The LF speed only scales a dissipative term of the size of the stencil's
  fifth differences: on smooth data the two right-hand sides differ at
  O(h^5), and the solver still converges at fifth order.
* The global speeds are the largest |lambda^s| of a sweep: on a uniform
  state they are |v_n - c_f|, |v_n - c_A|, ... of that state."""
import math

import numpy as np
import pytest

from paper_1808_10633_amd import inputs as I


def test_two_state_data_gives_identical_rhs(orc):
    for gamma, u, n in ((2.0, I.brio_wu(64), 64), (1.4, I.sod(64), 64)):
        g = orc.Grid(n, dx=1.0 / n, gamma=gamma, bc=(1, 1, 0, 0, 0, 0))
        r0 = orc.rhs(g, u)
        g.lf_global = 1
        r1 = orc.rhs(g, u)
        assert np.array_equal(r0, r1)


def test_rhs_gap_closes_at_fifth_order(orc):
    gaps = []
    for n in (32, 64, 128):
        u, _ = I.linear_wave_1d("fast", n, amp=0.1)
        g = orc.Grid(n, dx=1.0 / n)
        r0 = orc.rhs(g, u)
        g.lf_global = 1
        gaps.append(np.abs(orc.rhs(g, u) - r0).max())
    order = np.log2(np.array(gaps[:-1]) / np.array(gaps[1:]))
    assert (order > 4.5).all(), (gaps, order)


@pytest.mark.parametrize("family,amp", [("alfven", 1e-5), ("entropy", 1e-5), ("fast", 1e-7)])
def test_linear_wave_fifth_order_with_global_speeds(orc, family, amp):
    errs = []
    for n in (16, 32, 64):
        u, speed = I.linear_wave_1d(family, n, amp=amp)
        g = orc.Grid(n, dx=1.0 / n, cfl=0.4, lf_global=1)
        T, t = 1.0 / abs(speed), 0.0
        while t < T - 1e-14:
            dt = min(orc.cfl_dt(g, u), T - t)
            orc.rk4_step(g, u, dt)
            t += dt
        ue, _ = I.linear_wave_1d(family, n, amp=amp, t=T)
        e = np.abs(g.interior(u) - g.interior(ue)).mean(axis=(1, 2, 3))
        errs.append(math.sqrt((e ** 2).sum()))
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert (order > 4.7).all(), (errs, order)


def test_global_speeds_of_a_uniform_state(orc):
    # rho = 1.3, v = (0.4, -0.2, 0.1), B = (0.6, 0.3, -0.5), p = 0.9 in 3-D:
    # along x, c_A = |B_x|/sqrt(rho) and c_f, c_s from the textbook roots
    rho, v, B, p, gam = 1.3, np.array([0.4, -0.2, 0.1]), np.array([0.6, 0.3, -0.5]), 0.9, 5.0 / 3.0
    g = orc.Grid(6, 5, 4, 0.1, 0.1, 0.1)
    u = np.zeros(g.shape)
    g.interior(u)[...] = orc.prim_to_cons(np.array([rho, *v, *B, p]), gam)[:, None, None, None]
    orc.fill_ghosts(g, u)
    for d in range(3):
        a2 = gam * p / rho
        b2 = B @ B / rho
        bn2 = B[d] ** 2 / rho
        root = math.sqrt((a2 + b2) ** 2 - 4 * a2 * bn2)
        cf, cs, ca = math.sqrt(0.5 * (a2 + b2 + root)), math.sqrt(0.5 * (a2 + b2 - root)), math.sqrt(bn2)
        vn = v[d]
        want = np.abs([vn - cf, vn - ca, vn - cs, vn, vn + cs, vn + ca, vn + cf])
        assert np.allclose(orc.lf_global(g, u, d), want, rtol=1e-13, atol=0)
