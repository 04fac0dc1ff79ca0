"""Exact moving solutions of ideal MHD as pins of the oracle (1-D, outflow
ends, fronts kept away from the ends): closed forms, not the oracle's code.

* Contact discontinuity: a density jump in uniform v, p, B is carried at v_x;
  velocity, pressure and field stay uniform.
* Rotational discontinuity: the transverse field turns by an angle across the
  front at fixed |B_t|, with v_t = -B_t / sqrt(rho) (for B_x > 0); the front
  moves at v_x + B_x / sqrt(rho).
* Perpendicular fast shock: the downstream state follows from the
  Rankine-Hugoniot relations (mass, momentum, flux freezing, energy; the
  compression ratio found here by bisection); with the upstream gas at rest
  the shock moves at the upstream inflow speed of the shock frame.
The front of each is located where a monotone variable crosses the mean of
its two states, and must sit within one cell of the exact position."""
import math

import numpy as np

from paper_1808_10633_amd import inputs as I

G53 = 5.0 / 3.0


def _tube(orc, n, WL, WR, gamma=G53, x0=0.5):
    u = I._tube(n, WL, WR, gamma, x0=x0)
    g = orc.Grid(n, dx=1.0 / n, gamma=gamma, bc=(1, 1, 0, 0, 0, 0))
    return g, u


def _run(orc, g, u, T):
    t = 0.0
    while t < T - 1e-14:
        dt = min(orc.cfl_dt(g, u), T - t)
        orc.rk4_step(g, u, dt)
        t += dt


def _front(q, n):
    """x where the monotone profile q (cell centres (i + 1/2)/n) crosses the
    mean of its end values, by linear interpolation."""
    mid = 0.5 * (q[0] + q[-1])
    s = np.sign(q - mid)
    i = int(np.nonzero(s[:-1] * s[1:] <= 0)[0][0])
    x = (np.arange(n) + 0.5) / n
    return x[i] + (mid - q[i]) / (q[i + 1] - q[i]) * (x[i + 1] - x[i])


def test_contact_discontinuity_translates_at_vx(orc):
    n, vx, T = 200, 0.4, 0.5
    WL = (2.0, vx, -0.3, 0.2, 0.7, 0.5, -0.4, 1.2)
    WR = (0.5, vx, -0.3, 0.2, 0.7, 0.5, -0.4, 1.2)
    g, u = _tube(orc, n, WL, WR, x0=0.3)
    _run(orc, g, u, T)
    w = g.interior(u)[:, 0, 0]
    rho = w[0]
    assert abs(_front(rho, n) - (0.3 + vx * T)) < 1.0 / n
    v = w[1:4] / rho
    p = (G53 - 1) * (w[7] - 0.5 * (w[1:4] ** 2).sum(0) / rho - 0.5 * (w[4:7] ** 2).sum(0))
    assert np.abs(v - np.array(WL[1:4])[:, None]).max() < 1e-10
    assert np.abs(p - 1.2).max() < 1e-10
    assert np.abs(w[4:7] - np.array(WL[4:7])[:, None]).max() < 1e-12


def test_rotational_discontinuity_moves_at_alfven_speed(orc):
    # T = 0.1: the fast waves the smeared front sheds (speed v_x -+ c_f,
    # c_f ~ 1.8) stay inside the tube
    n, T = 200, 0.1
    rho, p, vx, bx, bt, theta = 1.0, 1.0, 0.2, 1.0, 0.8, 0.5 * math.pi
    def state(angle):
        by, bz = bt * math.cos(angle), bt * math.sin(angle)
        return (rho, vx, -by / math.sqrt(rho), -bz / math.sqrt(rho), bx, by, bz, p)
    g, u = _tube(orc, n, state(0.0), state(theta), x0=0.5)
    _run(orc, g, u, T)
    w = g.interior(u)[:, 0, 0]
    ang = np.unwrap(np.arctan2(w[6], w[5]))            # angle of B_t, monotone across the front
    ca = bx / math.sqrt(rho)
    assert abs(_front(ang, n) - (0.5 + (vx + ca) * T)) < 1.0 / n
    # the far states keep their values (the smeared front sheds compressive
    # waves of a few per cent in rho and p: numerical, not part of the exact
    # solution, so not pinned)
    assert abs(ang[0]) < 1e-12 and abs(ang[-1] - theta) < 1e-12
    bmag = np.hypot(w[5], w[6])
    assert abs(bmag[0] - bt) < 1e-12 and abs(bmag[-1] - bt) < 1e-12


def _perpendicular_shock(rho1, p1, b1, w, gamma):
    """Downstream state of a perpendicular shock (B normal to the shock
    normal) in the shock frame, for upstream inflow speed w toward the shock:
    mass rho1 w = rho2 w2, flux freezing b1 w = b2 w2, momentum
    rho1 w^2 + p1 + b1^2/2 = rho2 w2^2 + p2 + b2^2/2 and energy
    (rho w^2/2 + gamma p/(gamma-1) + b^2) w conserved; the compression
    r = rho2/rho1 solves the energy relation (bisection on (1, (gamma+1)/(gamma-1)))."""
    def resid(r):
        w2, b2 = w / r, b1 * r
        p2 = p1 + 0.5 * b1 ** 2 + rho1 * w ** 2 - rho1 * r * w2 ** 2 - 0.5 * b2 ** 2
        f1 = (0.5 * rho1 * w ** 2 + gamma * p1 / (gamma - 1) + b1 ** 2) * w
        f2 = (0.5 * rho1 * r * w2 ** 2 + gamma * p2 / (gamma - 1) + b2 ** 2) * w2
        return f2 - f1, p2
    lo, hi = 1.0 + 1e-9, (gamma + 1) / (gamma - 1) - 1e-9
    assert resid(lo)[0] * resid(hi)[0] < 0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if resid(lo)[0] * resid(mid)[0] <= 0:
            hi = mid
        else:
            lo = mid
    r = 0.5 * (lo + hi)
    return r, resid(r)[1]


def test_perpendicular_fast_shock_speed(orc):
    n, T, gamma = 400, 0.15, G53
    rho1, p1, b1 = 1.0, 1.0, 1.0
    cf = math.sqrt((gamma * p1 + b1 ** 2) / rho1)
    w = 2.0 * cf                                             # fast Mach 2
    r, p2 = _perpendicular_shock(rho1, p1, b1, w, gamma)
    assert 1.0 < r < 4.0 and p2 > p1
    v2 = w * (1.0 - 1.0 / r)                                  # lab frame: upstream at rest
    WL = (rho1 * r, v2, 0.0, 0.0, 0.0, b1 * r, 0.0, p2)      # downstream (left)
    WR = (rho1, 0.0, 0.0, 0.0, 0.0, b1, 0.0, p1)              # upstream (right)
    g, u = _tube(orc, n, WL, WR, gamma=gamma, x0=0.25)
    _run(orc, g, u, T)
    rho = g.interior(u)[0, 0, 0]
    assert abs(_front(rho, n) - (0.25 + w * T)) < 1.0 / n
    # the upstream plateau is untouched and the downstream one holds its
    # Rankine-Hugoniot value up to the start-up error of a captured shock
    # (waves shed while the sharp initial jump becomes a discrete shock)
    assert abs(rho[n // 8] - rho1 * r) < 1e-4 * r and abs(rho[-n // 8] - rho1) < 1e-12
