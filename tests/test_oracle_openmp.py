"""The OpenMP build of the oracle (the all-core CPU baseline) computes the
same numbers as the serial build: the pragmas only share the independent
k-plane loops among threads, so every value comes out of the same code and
the two builds agree bit for bit."""
import numpy as np

from paper_1808_10633_amd import inputs as I


def test_openmp_build_matches_serial_bitwise(orc):
    n = 10
    g = orc.Grid(n, n, n, 1.0 / n, 1.0 / n, 1.0 / n)
    u = I.turbulence((n, n, n), mach=1.0, beta=10.0, seed=21, kmax=4).numpy().copy()
    try:
        assert orc.set_threads(1) == 1
        r1 = orc.rhs(g, u)
        s1 = u.copy()
        dt = orc.cfl_dt(g, s1)
        orc.rk4_step(g, s1, dt)
        used = orc.set_threads(4)
        assert used == 4
        r4 = orc.rhs(g, u)
        s4 = u.copy()
        assert orc.cfl_dt(g, s4) == dt
        orc.rk4_step(g, s4, dt)
    finally:
        orc.set_threads(1)
    assert np.array_equal(r1, r4)
    assert np.array_equal(s1, s4)
    # a 2-D outflow box exercises the inactive axis and the other faces
    g2 = orc.Grid(12, 9, 1, 1 / 12, 1 / 9, 1.0, bc=(1, 1, 0, 0, 0, 0))
    rng = np.random.default_rng(5)
    sh = g2.shape[1:]
    rho = 1 + 0.2 * rng.uniform(size=sh)
    v = 0.3 * rng.normal(size=(3,) + sh)
    B = 0.5 * rng.normal(size=(3,) + sh)
    p = 1 + 0.2 * rng.uniform(size=sh)
    u2 = np.concatenate([rho[None], rho * v, B,
                         (p / (g2.gamma - 1) + 0.5 * rho * (v ** 2).sum(0) + 0.5 * (B ** 2).sum(0))[None]])
    u2 = np.ascontiguousarray(u2)
    try:
        orc.set_threads(1)
        a = orc.rhs(g2, u2)
        orc.set_threads(3)
        b = orc.rhs(g2, u2)
    finally:
        orc.set_threads(1)
    assert np.array_equal(a, b)
