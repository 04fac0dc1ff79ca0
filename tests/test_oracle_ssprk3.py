"""Pins of the oracle's SSP-RK3 step (Shu & Osher 1988), the ablation of the
classical RK4 that Sec. 2.1 of arXiv:1808.10633 uses: facts of the
integrator, not of the oracle's code.

* Third order in time: on a fixed grid, halving dt shrinks the difference
  between successive solutions by 2^3 (a wrong stage weight drops the order).
* It differs from RK4 by its own O(dt^3) error: the gap between the two
  shrinks by 2^3 per halving.
* A steady state (uniform flow, L(U) = 0) is a fixed point: each stage is a
  convex combination of copies of the same state.
* A Brio-Wu shock tube keeps positive density and pressure and, before the
  waves reach the outflow ends (where v = 0), conserves the quantities whose
  flux vanishes there: mass, m_z, B_y and energy."""
import numpy as np

from paper_1808_10633_amd import inputs as I


def _fixed_steps(orc, step, g, u, T, nsteps):
    for _ in range(nsteps):
        step(g, u, T / nsteps)
    return u


def test_ssprk3_third_order_in_time(orc):
    n = 24
    sols = []
    for nsteps in (8, 16, 32):
        u, _ = I.linear_wave_1d("fast", n, amp=1e-2)
        g = orc.Grid(n, dx=1.0 / n)
        _fixed_steps(orc, orc.ssprk3_step, g, u, 0.25, nsteps)
        sols.append(g.interior(u).copy())
    r = np.abs(sols[0] - sols[1]).max() / np.abs(sols[1] - sols[2]).max()
    assert 6.5 < r < 9.5, r


def test_ssprk3_differs_from_rk4_at_third_order(orc):
    n = 24
    gaps = []
    for nsteps in (8, 16, 32):
        a, _ = I.linear_wave_1d("fast", n, amp=1e-2)
        b = a.copy()
        g = orc.Grid(n, dx=1.0 / n)
        _fixed_steps(orc, orc.ssprk3_step, g, a, 0.25, nsteps)
        _fixed_steps(orc, orc.rk4_step, g, b, 0.25, nsteps)
        gaps.append(np.abs(g.interior(a) - g.interior(b)).max())
    r = np.array(gaps[:-1]) / np.array(gaps[1:])
    assert ((r > 6.5) & (r < 9.5)).all(), (gaps, r)


def test_ssprk3_steady_state_is_a_fixed_point(orc):
    g = orc.Grid(8, 7, 6, 1 / 8, 1 / 7, 1 / 6)
    u = np.zeros(g.shape)
    W0 = np.array([1.3, 0.2, -0.1, 0.3, 0.5, -0.4, 0.2, 0.8])
    g.interior(u)[...] = orc.prim_to_cons(W0)[:, None, None, None]
    ref = g.interior(u).copy()
    orc.ssprk3_step(g, u, 0.01)
    assert np.abs(g.interior(u) - ref).max() < 1e-15


def test_ssprk3_brio_wu_positive_and_conservative(orc):
    n = 200
    u = I.brio_wu(n)
    g = orc.Grid(n, dx=1.0 / n, gamma=2.0, bc=(1, 1, 0, 0, 0, 0))
    s0 = orc.sums(g, u)
    t = 0.0
    while t < 0.1:                       # the fast fans stay inside the tube until t ~ 0.25
        dt = orc.cfl_dt(g, u)
        orc.ssprk3_step(g, u, dt)
        t += dt
    w = g.interior(u)[:, 0, 0]
    p = (2.0 - 1.0) * (w[7] - 0.5 * (w[1] ** 2 + w[2] ** 2 + w[3] ** 2) / w[0]
                       - 0.5 * (w[4] ** 2 + w[5] ** 2 + w[6] ** 2))
    assert w[0].min() > 0.1 and p.min() > 0.05
    s1 = orc.sums(g, u)
    # rho, m_z, B_y, E: zero flux through the still ends (v = 0 there up to the
    # round-off that the nonlinear weights carry across the tube)
    for v in (0, 3, 5, 7):
        assert abs(s1[v] - s0[v]) < 1e-11 * np.abs(w[v]).sum() + 1e-300, (v, s0[v], s1[v])
