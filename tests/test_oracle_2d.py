"""The oracle on the 2-D problems of Sec. 3.1 (Orszag-Tang vortex,
Kelvin-Helmholtz instability): facts of the equations, not of the code.

* A planar flow stays planar: with no component and no gradient along z,
  the z momentum and z field stay exactly zero (and B = 0 stays zero).
* The Orszag-Tang state is symmetric under the point reflection
  (x, y) -> (-x, -y) with v and B odd; the equations, and a scheme whose
  flux is mirror-symmetric, keep that symmetry.
* Mass, momentum, energy and field are conserved on the periodic box, and
  the corner divergence of B stays at its initial zero.
* The Kelvin-Helmholtz perturbation grows: the vertical kinetic energy rises
  many-fold while the shear layers roll up."""
import numpy as np

from paper_1808_10633_amd import inputs as I

ODD = np.array([1, -1, -1, -1, -1, -1, -1, 1])[:, None, None]


def _run(orc, g, u, T=None, steps=None):
    t, s = 0.0, 0
    while (T is not None and t < T - 1e-14) or (steps is not None and s < steps):
        dt = orc.cfl_dt(g, u)
        if T is not None:
            dt = min(dt, T - t)
        orc.rk4_step(g, u, dt)
        t += dt
        s += 1
    return t


def test_orszag_tang_symmetry_planarity_conservation(orc):
    n = 32                                   # a power of two: cell centres mirror exactly
    u = I.orszag_tang(n)
    g = orc.Grid(n, n, 1, 1.0 / n, 1.0 / n, 1.0)
    v0 = g.interior(u)[:, 0].copy()
    assert np.abs(v0 - ODD * v0[:, ::-1, ::-1]).max() == 0.0     # the set-up is exactly symmetric
    s0 = np.array(orc.sums(g, u))
    _run(orc, g, u, T=0.25)                  # shocks have formed by t = 0.25
    v = g.interior(u)[:, 0]
    scale = np.array([v[0].max()] + [np.abs(v[1:4]).max()] * 3 + [np.abs(v[4:7]).max()] * 3 + [v[7].max()])
    sym = (np.abs(v - ODD * v[:, ::-1, ::-1]).max(axis=(1, 2)) / scale).max()
    assert sym < 1e-13, sym
    assert np.abs(v[3]).max() == 0.0 and np.abs(v[6]).max() == 0.0      # m_z, B_z
    ds = np.abs(np.array(orc.sums(g, u)) - s0)
    assert (ds <= 1e-13 * np.abs(v0).reshape(8, -1).sum(axis=1).clip(1.0)).all(), ds
    mx, _ = orc.divb(g, u)
    assert mx < 1e-12 * np.abs(v[4:6]).max() * n


def test_kelvin_helmholtz_planar_and_growing(orc):
    n = 16
    u = I.kelvin_helmholtz(n)
    g = orc.Grid(n, 2 * n, 1, 1.0 / n, 1.0 / n, 1.0)
    sl = I.interior_slices(n, 2 * n, 1)

    def ez():
        w = u[sl][:, 0]
        return float((0.5 * w[2] ** 2 / w[0]).mean())

    e0 = ez()
    s0 = np.array(orc.sums(g, u))
    _run(orc, g, u, T=1.5)
    w = u[sl][:, 0]
    assert np.abs(w[3]).max() == 0.0 and np.abs(w[4:7]).max() == 0.0   # m_z = 0, B = 0 exactly
    assert ez() > 20 * e0, (ez(), e0)
    ds = np.abs(np.array(orc.sums(g, u)) - s0)
    assert ds[0] < 1e-12 * abs(s0[0]) and ds[7] < 1e-12 * abs(s0[7])
