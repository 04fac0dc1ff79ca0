"""Staggered face-B storage (the CT ablation of Sec. 2.1: constrained
transport on a staggered mesh after Ryu et al.): the B slots hold the normal
field of each cell's lower face, the sweeps see the mean of a cell's two
faces, and each face advances by -(curl E).n from the same edge EMFs.

Pins:
* the face divergence of a field built from an edge vector potential stays
  at round-off over several steps (the staggered form's own invariant);
* the form is the cell-centred scheme with B_cell = mean of the faces: from
  matching states the two give the same cell fields, time steps and hydro
  variables to round-off (every face update is linear in the same EMFs);
* on the inclined Alfven wave the face field converges to the exact
  travelling wave at second order, as CT limits it (Sec. 2.1).
"""
import numpy as np

from paper_1808_10633_amd import inputs as I


def _grids(orc, n):
    h = 1.0 / n
    return orc.Grid(n, n, n, h, h, h), orc.Grid(n, n, n, h, h, h, b_face=1)


def _face_div(u, n):
    """Face divergence field of a periodic staggered state (interior), in
    units of 1/dx: sum_d (slot_d(i + e_d) - slot_d(i)) with periodic wrap."""
    b = u[4:7, 3:3 + n, 3:3 + n, 3:3 + n]
    return sum(np.roll(b[d], -1, axis=2 - d) - b[d] for d in range(3)) * n


def test_face_divergence_is_invariant(orc):
    n = 12
    gc, gf = _grids(orc, n)
    u = I.turbulence((n, n, n), mach=1.5, beta=1.0, seed=41, kmax=4, b_faces=True).numpy().copy()
    bmax = np.abs(gf.interior(u)[4:7]).max()
    d0, _ = orc.divb_face(gf, u)
    assert d0 < 1e-13 * bmax * n
    # a divergence planted on a few faces: divb_face reads it, and the
    # evolution keeps the divergence field of every cell unchanged
    w = u.copy()
    w[4, 3 + 5, 3 + 2, 3 + 7] += 1e-3
    w[5, 3 + 1, 3 + 9, 3 + 0] -= 2e-3
    div0 = _face_div(w, n)
    assert abs(orc.divb_face(gf, w)[0] - np.abs(div0).max()) < 1e-12 * np.abs(div0).max()
    for _ in range(3):
        dt = orc.cfl_dt(gf, u)
        orc.rk4_step(gf, u, dt)
        orc.rk4_step(gf, w, dt)
    d1, _ = orc.divb_face(gf, u)
    assert d1 < 1e-13 * bmax * n, (d0, d1)
    div1 = _face_div(w, n)
    assert np.abs(div1 - div0).max() < 1e-13 * bmax * n
    assert np.abs(div1).max() > 0.5 * 2e-3 * n


def test_staggered_form_equals_cell_form_with_face_means(orc):
    n = 12
    gc, gf = _grids(orc, n)
    uf = I.turbulence((n, n, n), mach=1.5, beta=1.0, seed=42, kmax=4, b_faces=True).numpy().copy()
    uc = orc.face_to_cell(gf, uf)
    assert orc.cfl_dt(gf, uf) == orc.cfl_dt(gc, uc)
    for _ in range(3):
        dtf = orc.cfl_dt(gf, uf)
        dtc = orc.cfl_dt(gc, uc)
        assert abs(dtf - dtc) <= 1e-14 * dtc
        orc.rk4_step(gf, uf, dtf)
        orc.rk4_step(gc, uc, dtf)
    a = gc.interior(orc.face_to_cell(gf, uf))
    b = gc.interior(uc)
    scale = np.abs(b).reshape(8, -1).max(axis=1)[:, None, None, None]
    err = np.abs(a - b) / scale
    assert err.max() < 1e-13, err.reshape(8, -1).max(axis=1)
    # rho, m, E are the same variables in both forms
    assert np.abs(gf.interior(uf)[[0, 1, 2, 3, 7]] - b[[0, 1, 2, 3, 7]]).max() < 1e-13 * np.abs(b).max()


def test_staggered_alfven_wave_converges_at_second_order(orc):
    errs = []
    for n in (8, 16):
        _, gf = _grids(orc, n)
        u, _ = I.alfven_wave_3d(n, b_faces=True)
        T = 0.02
        t = 0.0
        while t < T - 1e-15:
            dt = min(orc.cfl_dt(gf, u), T - t)
            orc.rk4_step(gf, u, dt)
            t += dt
        ue, _ = I.alfven_wave_3d(n, t=T, b_faces=True)
        errs.append(np.abs(gf.interior(u)[4:7] - gf.interior(ue)[4:7]).max())
        assert orc.divb_face(gf, u)[0] < 1e-12
    assert errs[1] < errs[0] / 3.5 and errs[1] < 1e-8, errs
