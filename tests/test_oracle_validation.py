"""The oracle against a number the paper prints: field-loop advection
(Sec. 3.1), magnetic energy kept at t = 1 by WENO5 at 64 zones (about 95 %)."""
import os

import numpy as np
import pytest

from paper_1808_10633_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "field_loop_energy.txt")


@pytest.mark.slow
def test_oracle_field_loop_energy(orc):
    vals = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    n = 32                                    # 64 zones along x: a 64 x 32 box
    u = I.field_loop(n)
    g = orc.Grid(2 * n, n, 1, 2.0 / (2 * n), 1.0 / n, 1.0)
    sl = I.interior_slices(2 * n, n, 1)
    e0 = float((u[sl][4] ** 2 + u[sl][5] ** 2).sum())
    t = 0.0
    while t < vals["time"] - 1e-12:
        orc.fill_ghosts(g, u)
        dt = min(orc.cfl_dt(g, u), vals["time"] - t)
        orc.rk4_step(g, u, dt)
        t += dt
    frac = float((u[sl][4] ** 2 + u[sl][5] ** 2).sum()) / e0
    # the paper's value is read off a figure; 64 zones along y (a 128 x 64 box,
    # too slow here) keeps more: the two readings bracket it
    assert abs(frac - vals["energy_fraction"]) < 0.03, frac
    assert frac < 1.0
