"""Seeded synthetic initial conditions for the WENO5-MHD stage.

These generators feed both the GPU library and the CPU oracle; they contain
none of the scheme's arithmetic (no WENO, no characteristic projection, no CT,
no time stepping).  Every state is returned as the padded conserved array
``u[v][k][j][i]`` with ``v = (rho, mx, my, mz, Bx, By, Bz, E)``, 3 ghost cells
per side on every axis with more than one cell (0 on an inactive axis), the
interior holding point values at cell centres ``x_i = (i + 1/2) dx``.  Ghost
cells are left at zero; the solvers fill them.

Workloads (the paper's own test problems are analytic, Sec. 3.1):
  * ``alfven_wave_3d``: a small-amplitude Alfven wave travelling along the grid
    diagonal of a periodic cube, background B0 = (1, sqrt2, 1/2)/|.| in the
    wave frame, rho = 1, p = 1/gamma.
  * ``linear_wave_1d``: one of the four MHD linear waves (fast, Alfven, slow,
    entropy) on a 1-D periodic line, after the convergence test of Sec. 3.1.
  * ``turbulence``: decaying MHD turbulence: random Gaussian Fourier modes with
    2 <= |k|/2pi <= 8 and |v_k|^2 ~ k^-11/3, solenoidal (optionally with a
    compressive share), a uniform seed field plus a random field from an edge
    vector potential (so its corner divergence vanishes), optional log-normal
    density.
  * ``sod``, ``brio_wu``: 1-D shock tubes.
  * ``field_loop``, ``orszag_tang``, ``kelvin_helmholtz``: the 2-D problems of
    Sec. 3.1 (field-loop advection, the Orszag-Tang vortex, a Kelvin-Helmholtz
    instability with the printed parameters).
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 5.0 / 3.0


def ghosts(nx, ny, nz):
    return tuple(3 if n > 1 else 0 for n in (nx, ny, nz))


def padded_shape(nx, ny, nz):
    gx, gy, gz = ghosts(nx, ny, nz)
    return (8, nz + 2 * gz, ny + 2 * gy, nx + 2 * gx)


def interior_slices(nx, ny, nz):
    gx, gy, gz = ghosts(nx, ny, nz)
    return (slice(None), slice(gz, gz + nz), slice(gy, gy + ny), slice(gx, gx + nx))


def conserved(rho, v, B, p, gamma):
    """Conserved variables from primitive fields (ideal gas, B^2/2 pressure)."""
    xp = np
    try:
        import torch
        if isinstance(rho, torch.Tensor):
            xp = torch
    except ImportError:  # pragma: no cover
        pass
    kin = 0.5 * rho * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
    mag = 0.5 * (B[0] ** 2 + B[1] ** 2 + B[2] ** 2)
    E = p / (gamma - 1.0) + kin + mag
    return xp.stack([rho, rho * v[0], rho * v[1], rho * v[2], B[0], B[1], B[2], E])


def _pad(interior, nx, ny, nz):
    out = np.zeros(padded_shape(nx, ny, nz))
    out[interior_slices(nx, ny, nz)] = interior
    return out


def cell_centres(n, d=None):
    d = 1.0 / n if d is None else d
    return (np.arange(n) + 0.5) * d


# --------------------------------------------------------------------------
# Linear waves
# --------------------------------------------------------------------------

def alfven_background(gamma=GAMMA):
    """Wave-frame background of the inclined Alfven-wave problem."""
    b = np.array([1.0, math.sqrt(2.0), 0.5])
    b = b / np.linalg.norm(b)
    return 1.0, 1.0 / gamma, b


def wave_frame():
    e1 = np.array([1.0, 1.0, 1.0]) / math.sqrt(3.0)
    e2 = np.array([-1.0, 1.0, 0.0]) / math.sqrt(2.0)
    e3 = np.cross(e1, e2)
    return e1, e2, e3


def alfven_wave_3d(n, amp=1e-6, gamma=GAMMA, t=0.0, b_faces=False):
    """Alfven wave along (1,1,1) in the periodic unit cube, n^3 cells.

    The wave has one wavelength per unit length along each axis
    (k = 2 pi (1,1,1)); it is the exact linear solution shifted by c_A t.
    b_faces: the B slots hold the field sampled at each cell's lower faces
    (staggered storage; E uses the mean of the two faces of a cell); the
    sampled face field has zero face divergence, as k . dB = 0 with equal
    wavenumbers on every axis.
    Returns (padded conserved state, Alfven speed).
    """
    rho0, p0, bw = alfven_background(gamma)
    e1, e2, e3 = wave_frame()
    B0 = bw[0] * e1 + bw[1] * e2 + bw[2] * e3
    bt = np.array([bw[1], bw[2]]) / np.hypot(bw[1], bw[2])
    # perturbation direction in the wave frame: perpendicular to k and B0
    dBdir = -bt[1] * e2 + bt[0] * e3
    ca = abs(bw[0]) / math.sqrt(rho0)
    x = cell_centres(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    phase = 2.0 * math.pi * (X + Y + Z - math.sqrt(3.0) * ca * t)
    c = amp * np.cos(phase)
    # right-going Alfven wave: dv = -sign(B_par) dB / sqrt(rho)
    s = 1.0 if bw[0] >= 0 else -1.0
    B = [B0[d] + c * math.sqrt(rho0) * dBdir[d] for d in range(3)]
    v = [-s * c * dBdir[d] for d in range(3)]
    rho = np.full_like(X, rho0)
    p = np.full_like(X, p0)
    if not b_faces:
        u = conserved(rho, v, B, p, gamma)
        return _pad(u, n, n, n), ca
    # lower faces of axis d sit half a cell below the centres along d
    h = 0.5 / n
    cf = amp * np.cos(phase - 2.0 * math.pi * h)       # the phase moves by -2 pi h along any one axis
    Bf = [B0[d] + cf * math.sqrt(rho0) * dBdir[d] for d in range(3)]
    Bc = [0.5 * (Bf[d] + np.roll(Bf[d], -1, axis=2 - d)) for d in range(3)]
    u = conserved(rho, v, Bc, p, gamma)
    u[4:7] = np.stack(Bf)
    return _pad(u, n, n, n), ca


def _primitive_jacobian(rho, v, B, p, gamma):
    """1-D ideal-MHD primitive-variable coefficient matrix along x for
    w = (rho, vx, vy, vz, By, Bz, p); Bx is constant.  Used only to obtain
    the linear eigenmodes of the wave test problems."""
    vx = v[0]
    Bx, By, Bz = B
    A = np.zeros((7, 7))
    A[0, 0] = vx; A[0, 1] = rho
    A[1, 1] = vx; A[1, 4] = By / rho; A[1, 5] = Bz / rho; A[1, 6] = 1.0 / rho
    A[2, 2] = vx; A[2, 4] = -Bx / rho
    A[3, 3] = vx; A[3, 5] = -Bx / rho
    A[4, 1] = By; A[4, 2] = -Bx; A[4, 4] = vx
    A[5, 1] = Bz; A[5, 3] = -Bx; A[5, 5] = vx
    A[6, 1] = gamma * p; A[6, 6] = vx
    return A


LINEAR_WAVES = ("fast", "alfven", "slow", "entropy")


def linear_wave_1d(family, n, amp=1e-5, gamma=GAMMA, t=0.0):
    """Right-going linear wave on the periodic unit line (n cells), background
    rho=1, p=1/gamma, B=(1, sqrt2, 1/2), v=0 (v_x=1 for the entropy wave).
    Returns (padded conserved state, wave speed)."""
    rho0, p0 = 1.0, 1.0 / gamma
    B0 = np.array([1.0, math.sqrt(2.0), 0.5])
    v0 = np.array([1.0 if family == "entropy" else 0.0, 0.0, 0.0])
    A = _primitive_jacobian(rho0, v0, B0, p0, gamma)
    lam, vec = np.linalg.eig(A)
    lam = lam.real
    vec = vec.real
    order = np.argsort(lam)
    lam, vec = lam[order], vec[:, order]
    # ascending: fast-, alfven-, slow-, entropy, slow+, alfven+, fast+
    idx = {"fast": 6, "alfven": 5, "slow": 4, "entropy": 3}[family]
    if family == "entropy":
        r = np.zeros(7); r[0] = 1.0
        speed = v0[0]
    else:
        r = vec[:, idx]
        speed = lam[idx]
        r = r / np.abs(r).max()
        if r[np.argmax(np.abs(r))] < 0:
            r = -r
    x = cell_centres(n)
    c = amp * np.sin(2.0 * math.pi * (x - speed * t))
    rho = rho0 + c * r[0]
    v = [v0[0] + c * r[1], v0[1] + c * r[2], v0[2] + c * r[3]]
    B = [np.full_like(x, B0[0]), B0[1] + c * r[4], B0[2] + c * r[5]]
    p = p0 + c * r[6]
    u = conserved(rho, v, B, p, gamma)
    return _pad(u.reshape(8, 1, 1, n), n, 1, 1), speed


# --------------------------------------------------------------------------
# Shock tubes (1-D, along x)
# --------------------------------------------------------------------------

def _tube(n, left, right, gamma, x0=0.5):
    x = cell_centres(n)
    L = x < x0
    prim = [np.where(L, left[i], right[i]) for i in range(8)]
    rho, vx, vy, vz, Bx, By, Bz, p = prim
    u = conserved(rho, [vx, vy, vz], [Bx, By, Bz], p, gamma)
    return _pad(u.reshape(8, 1, 1, n), n, 1, 1)


def sod(n, gamma=1.4):
    """Sod shock tube with B = 0: (rho, p) = (1, 1) | (0.125, 0.1)."""
    return _tube(n, (1.0, 0, 0, 0, 0, 0, 0, 1.0), (0.125, 0, 0, 0, 0, 0, 0, 0.1), gamma)


def brio_wu(n, gamma=2.0):
    """Brio-Wu MHD shock tube: Bx = 0.75, By = +1 | -1."""
    return _tube(n, (1.0, 0, 0, 0, 0.75, 1.0, 0, 1.0),
                 (0.125, 0, 0, 0, 0.75, -1.0, 0, 0.1), gamma)


# --------------------------------------------------------------------------
# Turbulence
# --------------------------------------------------------------------------

def _modes(dims, lengths, kmin, kmax):
    """Integer mode vectors m with kmin <= |m / L| <= kmax (k / 2pi)."""
    rng = [np.arange(-(n // 2) + 1, n // 2) if n > 1 else np.array([0]) for n in dims]
    M = np.stack(np.meshgrid(*rng, indexing="ij"), -1).reshape(-1, 3)
    kk = M / np.asarray(lengths)[None, :]
    kn = np.linalg.norm(kk, axis=1)
    sel = (kn >= kmin - 1e-12) & (kn <= kmax + 1e-12)
    return M[sel], kk[sel], kn[sel]


def _draw(gen, nmodes, ncomp):
    re = gen.standard_normal((nmodes, ncomp))
    im = gen.standard_normal((nmodes, ncomp))
    return re + 1j * im


def _synth(coef, M, dims, shift, torch_mod, device):
    """Real field sum_m Re[coef_m exp(2 pi i m . x / n)] at positions
    x_d = i_d + shift_d (in cells), via one inverse FFT per component."""
    nx, ny, nz = dims
    ncomp = coef.shape[1]
    phase = np.exp(1j * math.pi * 2.0 * (M * np.asarray(shift)[None, :]
                                          / np.asarray(dims)[None, :]).sum(1))
    c = coef * phase[:, None]
    torch = torch_mod
    grid = torch.zeros((ncomp, nz, ny, nx), dtype=torch.complex128, device=device)
    iz = torch.as_tensor(M[:, 2] % nz, device=device)
    iy = torch.as_tensor(M[:, 1] % ny, device=device)
    ix = torch.as_tensor(M[:, 0] % nx, device=device)
    cc = torch.as_tensor(c.T.copy(), dtype=torch.complex128, device=device)
    for q in range(ncomp):
        grid[q].index_put_((iz, iy, ix), cc[q], accumulate=True)
    field = torch.fft.ifftn(grid, dim=(1, 2, 3)) * float(nx * ny * nz)
    return field.real.contiguous()


def turbulence(dims, mach, beta, seed, *, dx=None, gamma=GAMMA, rho0=1.0, p0=1.0,
               kmin=2.0, kmax=8.0, compressive_fraction=0.0, lognormal_sigma=0.0,
               device="cpu", dtype=None, b_faces=False):
    """Decaying MHD turbulence box (periodic), returned as a padded conserved
    torch tensor on ``device``.

    dims: (nx, ny, nz).  dx: cell width (default 1/nx, i.e. a unit box along x).
    Velocity: random Gaussian modes, amplitude |k|^(-11/6) (shell power
    ~ k^(-11/3)), projected solenoidal; ``compressive_fraction`` of the kinetic
    energy in the compressive part; rms speed mach * sqrt(gamma p0 / rho0).
    Field: uniform B0 x-hat with B0^2 = p0/beta plus a random part with
    <dB^2> = p0/beta from an edge-centred vector potential (amplitude
    |k|^(-17/6)); the discrete curl makes its corner divergence vanish.
    Density: uniform, or log-normal exp(sigma g - sigma^2/2) for a unit-variance
    random field g.  Pressure p0 uniform.  Seeds: velocity seed, field seed+1,
    density seed+2 (numpy PCG64).
    b_faces: the B slots hold the face fields themselves (slot d of a cell =
    the normal field of its lower d-face, zero face divergence), E the energy
    of the cell-centred field (the mean of the two faces, as without b_faces).
    """
    import torch
    nx, ny, nz = dims
    dx = 1.0 / nx if dx is None else dx
    lengths = (nx * dx, ny * dx, nz * dx)
    M, kk, kn = _modes(dims, lengths, kmin, kmax)
    nm = len(M)
    khat = kk / kn[:, None]
    dtype = torch.float64 if dtype is None else dtype
    cs = math.sqrt(gamma * p0 / rho0)

    def rms(f):
        return float(torch.sqrt((f ** 2).sum(0).mean()))

    # velocity
    g = np.random.Generator(np.random.PCG64(seed))
    a = _draw(g, nm, 3) * (kn ** (-11.0 / 6.0))[:, None]
    along = (a * khat).sum(1)[:, None] * khat
    sol = a - along
    v = _synth(sol, M, dims, (0.5, 0.5, 0.5), torch, device)
    v = v / rms(v)
    if compressive_fraction > 0.0:
        vc = _synth(along, M, dims, (0.5, 0.5, 0.5), torch, device)
        vc = vc / rms(vc)
        v = math.sqrt(1.0 - compressive_fraction) * v + math.sqrt(compressive_fraction) * vc
        v = v / rms(v)
    v = v * (mach * cs)

    # magnetic field from an edge vector potential A; the discrete curl of a
    # mode gives face fields i (kt x A_hat) with kt_d = 2 sin(pi m_d/n_d)/dx,
    # and the mean of the two faces of a cell multiplies by cos(pi m_d/n_d).
    g = np.random.Generator(np.random.PCG64(seed + 1))
    Ah = _draw(g, nm, 3) * (kn ** (-17.0 / 6.0))[:, None]
    th = math.pi * M / np.asarray(dims)[None, :]
    kt = 2.0 * np.sin(th) / dx
    cosf = np.cos(th)
    curl = 1j * np.cross(kt, Ah) * cosf
    dB = _synth(curl, M, dims, (0.5, 0.5, 0.5), torch, device)
    brms = math.sqrt(p0 / beta)
    scale = brms / rms(dB)
    dB = dB * scale
    B0 = math.sqrt(p0 / beta)
    B = [dB[0] + B0, dB[1], dB[2]]
    if b_faces:
        # component d at the lower d-faces (shift 0 along d), same modes and scale
        facec = 1j * np.cross(kt, Ah)
        Bf = []
        for d in range(3):
            sh = tuple(0.0 if e == d and dims[e] > 1 else 0.5 for e in range(3))
            Bf.append(_synth(facec[:, d:d + 1] * (cosf[:, d:d + 1] if dims[d] == 1 else 1.0), M, dims, sh, torch,
                             device)[0] * scale + (B0 if d == 0 else 0.0))

    if lognormal_sigma > 0.0:
        g = np.random.Generator(np.random.PCG64(seed + 2))
        s = _draw(g, nm, 1) * (kn ** (-11.0 / 6.0))[:, None]
        gf = _synth(s, M, dims, (0.5, 0.5, 0.5), torch, device)[0]
        gf = (gf - gf.mean()) / gf.std()
        rho = torch.exp(lognormal_sigma * gf - 0.5 * lognormal_sigma ** 2)
    else:
        rho = torch.full((nz, ny, nx), rho0, dtype=torch.float64, device=device)
    p = torch.full_like(rho, p0)
    u = conserved(rho, [v[0], v[1], v[2]], B, p, gamma)
    if b_faces:
        u[4:7] = torch.stack(Bf)
    out = torch.zeros(padded_shape(nx, ny, nz), dtype=torch.float64, device=device)
    out[interior_slices(nx, ny, nz)] = u
    return out.to(dtype)


def field_loop(n, gamma=GAMMA, amp=1e-3, radius=0.3, v=(2.0, 1.0)):
    """Field-loop advection (the magnetic-energy test of Sec. 3.1): a 2n x n
    periodic box [-1, 1] x [-1/2, 1/2], rho = 1, p = 1, uniform velocity v
    (after t = 1 the loop is back where it started), and a weak loop from
    the potential A_z = amp (radius - r) inside r < radius.  A_z is sampled
    at cell corners; the face fields are its discrete curl and the cell
    field their two-face mean, so the corner divergence of the cell field
    vanishes.  Returns a padded numpy array (8, 1, n + 6, 2n + 6)."""
    nx, ny = 2 * n, n
    dx = 2.0 / nx
    dy = 1.0 / ny
    xc = -1.0 + dx * np.arange(nx + 1)           # corners
    yc = -0.5 + dy * np.arange(ny + 1)
    X, Y = np.meshgrid(xc, yc, indexing="xy")     # (ny+1, nx+1)
    r = np.sqrt(X ** 2 + Y ** 2)
    A = np.where(r < radius, amp * (radius - r), 0.0)
    bx, by = _curl_from_corner_potential(A, dx, dy)
    rho = np.ones((ny, nx))
    z = np.zeros((ny, nx))
    U = conserved(rho, [z + v[0], z + v[1], z], [bx, by, z], np.ones((ny, nx)), gamma)
    return _pad(U[:, None, :, :], nx, ny, 1)


def _curl_from_corner_potential(A, dx, dy):
    """Cell-centred (Bx, By) of the field whose potential A_z is sampled at
    the (ny+1, nx+1) cell corners: face fields are the discrete curl and the
    cell field is the mean of its two faces, so the corner divergence of the
    cell field vanishes."""
    bx_face = (A[1:, :] - A[:-1, :]) / dy          # (ny, nx+1)
    by_face = -(A[:, 1:] - A[:, :-1]) / dx         # (ny+1, nx)
    return 0.5 * (bx_face[:, 1:] + bx_face[:, :-1]), 0.5 * (by_face[1:, :] + by_face[:-1, :])


def orszag_tang(n, gamma=GAMMA):
    """Orszag-Tang vortex (Sec. 3.1; the set-up of Stone et al. 2008 in
    Heaviside-Lorentz units): periodic [-1/2, 1/2]^2 with n x n cells,
    rho = 25/(36 pi), p = 5/(12 pi), v = (-sin 2 pi y, sin 2 pi x),
    B = B0 (-sin 2 pi y, sin 4 pi x) with B0 = 1/sqrt(4 pi), from the potential
    A_z = B0 (cos(4 pi x)/(4 pi) + cos(2 pi y)/(2 pi)) sampled at cell corners.
    The state is symmetric under the point reflection (x, y) -> (-x, -y)
    with v and B odd.  Returns a padded numpy array (8, 1, n + 6, n + 6)."""
    d = 1.0 / n
    xc = -0.5 + d * np.arange(n + 1)
    X, Y = np.meshgrid(xc, xc, indexing="xy")
    b0 = 1.0 / math.sqrt(4.0 * math.pi)
    A = b0 * (np.cos(4 * math.pi * X) / (4 * math.pi) + np.cos(2 * math.pi * Y) / (2 * math.pi))
    bx, by = _curl_from_corner_potential(A, d, d)
    x = -0.5 + d * (np.arange(n) + 0.5)
    Xc, Yc = np.meshgrid(x, x, indexing="xy")
    rho = np.full((n, n), 25.0 / (36.0 * math.pi))
    p = np.full((n, n), 5.0 / (12.0 * math.pi))
    z = np.zeros((n, n))
    U = conserved(rho, [-np.sin(2 * math.pi * Yc), np.sin(2 * math.pi * Xc), z], [bx, by, z], p, gamma)
    return _pad(U[:, None, :, :], n, n, 1)


def kelvin_helmholtz(nx, gamma=GAMMA, amp=0.01, p0=10.0, a=0.05, sigma=0.2, z1=0.5, z2=1.5,
                     u_flow=1.0, drho=1.0):
    """Kelvin-Helmholtz instability with the initial conditions of Lecoanet
    et al. (2016) and the parameters Sec. 3.1 prints (A = 0.01, P = 10,
    a = 0.05, sigma = 0.2, z1 = 0.5, z2 = 1.5, u_flow = 1, Delta rho = 1):
    periodic box [0, 1] x [0, 2] with nx x 2nx cells (the second axis plays
    z), B = 0,
      u_x = u_flow (tanh((z - z1)/a) - tanh((z - z2)/a) - 1),
      u_z = A sin(2 pi x) (exp(-(z - z1)^2/sigma^2) + exp(-(z - z2)^2/sigma^2)),
      rho = 1 + (Delta rho / 2) (tanh((z - z1)/a) - tanh((z - z2)/a)),  p = P.
    Returns a padded numpy array (8, 1, 2nx + 6, nx + 6)."""
    ny = 2 * nx
    d = 1.0 / nx
    x = d * (np.arange(nx) + 0.5)
    z = d * (np.arange(ny) + 0.5)
    X, Z = np.meshgrid(x, z, indexing="xy")       # (ny, nx)
    th = np.tanh((Z - z1) / a) - np.tanh((Z - z2) / a)
    ux = u_flow * (th - 1.0)
    uz = amp * np.sin(2 * math.pi * X) * (np.exp(-((Z - z1) / sigma) ** 2) + np.exp(-((Z - z2) / sigma) ** 2))
    rho = 1.0 + 0.5 * drho * th
    zero = np.zeros_like(X)
    U = conserved(rho, [ux, uz, zero], [zero, zero, zero], np.full_like(X, p0), gamma)
    return _pad(U[:, None, :, :], nx, ny, 1)
