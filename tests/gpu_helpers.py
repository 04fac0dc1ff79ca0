"""Shared helpers of the GPU parity tests (test code, not product code)."""
import math
import sys

import numpy as np

from paper_1808_10633_amd import inputs as I

G53 = 5.0 / 3.0


def say(*a):
    """Print and flush, so a failing GPU run names its case."""
    print(*a, flush=True)
    sys.stdout.flush()


def random_smooth(nx, ny, nz, seed, amp=0.1, B=(0.7, 0.4, -0.3), v=(0.2, -0.1, 0.15), gamma=G53):
    """Smooth random state: a few low Fourier modes per primitive field."""
    rng = np.random.default_rng(seed)
    x = [(np.arange(n) + 0.5) / n for n in (nx, ny, nz)]
    Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
    base = [1.0, *v, *B, 1.0]
    prim = []
    for q in range(8):
        f = np.full(X.shape, float(base[q]))
        for _ in range(3):
            k = rng.integers(-2, 3, size=3)
            k = np.where(np.array([nx, ny, nz]) > 1, k, 0)
            f = f + amp * rng.normal() * np.cos(2 * math.pi * (k[0] * X + k[1] * Y + k[2] * Z)
                                                + rng.uniform(0, 6))
        prim.append(f)
    rho, vx, vy, vz, bx, by, bz, p = prim
    u = I.conserved(rho, [vx, vy, vz], [bx, by, bz], p, gamma)
    out = np.zeros(I.padded_shape(nx, ny, nz))
    out[I.interior_slices(nx, ny, nz)] = u
    return out


def scaled_state_error(a, b, gamma=G53):
    """max_v max_cells |a-b| / S_v with S_rho = max rho, S_E = max E,
    S_m = max rho * max fast speed bound, S_B = max |B| (per-variable scales
    of the conserved state; a and b are interiors)."""
    rho = b[0]
    bb = b[4] ** 2 + b[5] ** 2 + b[6] ** 2
    p = (gamma - 1) * (b[7] - 0.5 * (b[1] ** 2 + b[2] ** 2 + b[3] ** 2) / rho - 0.5 * bb)
    cmax = math.sqrt(float((gamma * np.abs(p) / rho + bb / rho).max()))
    S = np.empty(8)
    S[0] = np.abs(rho).max()
    S[1:4] = np.abs(rho).max() * cmax
    S[4:7] = max(float(np.sqrt(b[4] ** 2 + b[5] ** 2 + b[6] ** 2).max()), 1e-300)
    S[7] = np.abs(b[7]).max()
    d = np.abs(a - b).reshape(8, -1).max(axis=1)
    return float((d / S).max()), d / S


def state_scales(u, gamma=G53):
    """Per-variable scales of a conserved state (interior): S_rho = max rho,
    S_m = max rho * c_max, S_B = max(max |B|, sqrt(max rho) c_max),
    S_E = max E, and c_max = max(|v| + sqrt(a^2 + b^2)) (bounds the fast
    speed)."""
    rho = u[0]
    bb = u[4] ** 2 + u[5] ** 2 + u[6] ** 2
    mm = u[1] ** 2 + u[2] ** 2 + u[3] ** 2
    p = (gamma - 1) * (u[7] - 0.5 * mm / rho - 0.5 * bb)
    cmax = float((np.sqrt(mm) / rho + np.sqrt((gamma * np.abs(p) + bb) / rho)).max())
    S = np.empty(8)
    S[0] = np.abs(rho).max()
    S[1:4] = S[0] * cmax
    S[4:7] = max(float(np.sqrt(bb).max()), math.sqrt(S[0]) * cmax)
    S[7] = np.abs(u[7]).max()
    return S, cmax


def scaled_rhs_error(a, b, u, dxmin):
    """Error of a right-hand side L(U), expressed as the state error it would
    cause over one CFL time dx_min / c_max: max_v max_cells |a-b| dt / S_v
    with the state scales of ``state_scales(u)``."""
    S, cmax = state_scales(u)
    dt = dxmin / cmax
    d = np.abs(a - b).reshape(8, -1).max(axis=1)
    return float((d * dt / S).max()), d * dt / S
