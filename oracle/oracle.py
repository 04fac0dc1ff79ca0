"""ctypes binding of the serial FP64 CPU oracle (``wombat_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline leg
of the benchmark use this module to check the GPU library; the product path
never imports it, and it imports nothing from the product package.

Method: Donnert et al., arXiv:1808.10633, Sec. 2.1 (characteristic WENO5
finite differences, eqs. 1-7, RK4, constrained transport) and Sec. 2.2
(3 ghost zones, x/y/z sweeps).  See the C source for the readings adopted
where the paper is silent.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wombat_oracle.c")
_LIB = os.path.join(_HERE, "libwombat_oracle.so")
_LIB_OMP = os.path.join(_HERE, "libwombat_oracle_omp.so")     # the same source with OpenMP

# No fast-math and no FMA contraction: every operation rounds as written.
CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = False, openmp: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/libwombat_oracle.so`` (with
    openmp: the same source with -fopenmp into ``libwombat_oracle_omp.so``)."""
    out = _LIB_OMP if openmp else _LIB
    srcs = (_SRC, os.path.join(_HERE, "wombat_oracle.h"))
    if force or not os.path.exists(out) or any(os.path.getmtime(out) < os.path.getmtime(f) for f in srcs):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, *(["-fopenmp"] if openmp else []), "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, out)
    return out


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("gamma", C.c_double), ("cfl", C.c_double), ("eps", C.c_double),
                ("bc", C.c_int * 6), ("weights", C.c_int), ("lf_global", C.c_int), ("b_face", C.c_int)]


@dataclass
class Grid:
    """Box description; an axis with n == 1 is inactive (no ghosts, no sweep)."""
    nx: int
    ny: int = 1
    nz: int = 1
    dx: float = 1.0
    dy: float = 1.0
    dz: float = 1.0
    gamma: float = 5.0 / 3.0
    cfl: float = 0.4
    eps: float = 1e-6
    bc: tuple = field(default_factory=lambda: (0, 0, 0, 0, 0, 0))   # 0 periodic, 1 outflow
    weights: int = 0          # 0: weights of eq. (3); 1: WENO-Z (ablation)
    lf_global: int = 0        # 0: LF speed per stencil; 1: per sweep over the box (ablation)
    b_face: int = 0           # 0: cell-centred B; 1: staggered face-normal B in the B slots (ablation)

    def c(self) -> _Grid:
        g = _Grid(self.nx, self.ny, self.nz, self.dx, self.dy, self.dz,
                  self.gamma, self.cfl, self.eps)
        for i in range(6):
            g.bc[i] = int(self.bc[i])
        g.weights = int(self.weights)
        g.lf_global = int(self.lf_global)
        g.b_face = int(self.b_face)
        return g

    @property
    def ghosts(self):
        return tuple(3 if n > 1 else 0 for n in (self.nx, self.ny, self.nz))

    @property
    def shape(self):
        """(8, NZ, NY, NX) padded state shape."""
        gx, gy, gz = self.ghosts
        return (8, self.nz + 2 * gz, self.ny + 2 * gy, self.nx + 2 * gx)

    def interior(self, u):
        gx, gy, gz = self.ghosts
        return u[:, gz:gz + self.nz, gy:gy + self.ny, gx:gx + self.nx]


_lib = None
_libs = {}
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def set_threads(n: int) -> int:
    """Route the oracle's calls to the serial build (n == 1) or to the OpenMP
    build of the same source with n host threads (n > 1).  Returns the
    threads in use."""
    global _lib
    key = "omp" if n > 1 else "serial"
    if key not in _libs:
        _libs[key] = _load(build(openmp=(key == "omp")))
    _lib = _libs[key]
    return int(_lib.orc_set_threads(int(n)))


def lib():
    global _lib
    if _lib is None:
        _lib = _libs["serial"] = _load(build())
    return _lib


def _load(path):
    L = C.CDLL(path)
    d = C.c_double
    L.orc_weno_weights.argtypes = [d, d, d, d, d, _dp, _dp]
    L.orc_weno_phi.argtypes = [d, d, d, d, d]
    L.orc_weno_weights_z.argtypes = [d, d, d, d, d, _dp, _dp]
    L.orc_interface_flux_z.argtypes = [_dp, d, d, _dp]
    L.orc_weno_phi.restype = d
    L.orc_weno_field_flux.argtypes = [_dp, _dp, d, d]
    L.orc_weno_field_flux.restype = d
    L.orc_weno_field_flux_z.argtypes = [_dp, _dp, d, d]
    L.orc_weno_field_flux_z.restype = d
    L.orc_prim_to_cons.argtypes = [_dp, d, _dp]
    L.orc_cons_to_prim.argtypes = [_dp, d, _dp]
    L.orc_flux.argtypes = [_dp, C.c_int, d, _dp]
    L.orc_wave_speeds.argtypes = [_dp, C.c_int, d, C.POINTER(d), C.POINTER(d), C.POINTER(d)]
    L.orc_eigensystem.argtypes = [_dp, d, _dp, _dp, _dp]
    L.orc_interface_flux.argtypes = [_dp, d, d, _dp]
    L.orc_interface_flux_ex.argtypes = [_dp, d, d, C.c_int, _dp, C.POINTER(d)]
    L.orc_linear_flux.argtypes = [_dp, d, _dp]
    g = C.POINTER(_Grid)
    L.orc_state_size.argtypes = [g]
    L.orc_state_size.restype = C.c_long
    L.orc_fill_ghosts.argtypes = [g, _dp]
    L.orc_rhs.argtypes = [g, _dp, _dp]
    L.orc_rhs.restype = C.c_int
    L.orc_rhs_nofill.argtypes = [g, _dp, _dp]
    L.orc_rhs_nofill.restype = C.c_int
    L.orc_rhs_linear.argtypes = [g, _dp, _dp]
    L.orc_rhs_linear.restype = C.c_int
    L.orc_cfl_dt.argtypes = [g, _dp]
    L.orc_cfl_dt.restype = d
    L.orc_rk4_step.argtypes = [g, _dp, d]
    L.orc_rk4_step.restype = C.c_int
    L.orc_ssprk3_step.argtypes = [g, _dp, d]
    L.orc_ssprk3_step.restype = C.c_int
    L.orc_lf_global.argtypes = [g, _dp, C.c_int, _dp]
    L.orc_interface_flux_alpha.argtypes = [_dp, d, d, C.c_int, _dp, _dp]
    L.orc_sums.argtypes = [g, _dp, _dp]
    L.orc_divb.argtypes = [g, _dp, C.POINTER(d), C.POINTER(d)]
    L.orc_face_to_cell.argtypes = [g, _dp, _dp]
    L.orc_divb_face.argtypes = [g, _dp, C.POINTER(d), C.POINTER(d)]
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_set_threads.restype = C.c_int
    return L


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---- scalar WENO (eqs. 1-7) ----
def weno_weights(a, b, c, d, eps=1e-6):
    w = np.zeros(3)
    s = np.zeros(3)
    lib().orc_weno_weights(a, b, c, d, eps, w, s)
    return w, s


def weno_weights_z(a, b, c, d, eps=1e-6):
    """WENO-Z weights (Borges et al. 2008, exponent 1): an ablation."""
    w = np.zeros(3)
    s = np.zeros(3)
    lib().orc_weno_weights_z(a, b, c, d, eps, w, s)
    return w, s


def weno_phi(a, b, c, d, eps=1e-6):
    return lib().orc_weno_phi(a, b, c, d, eps)


def weno_field_flux(f, u, alpha, eps=1e-6):
    return lib().orc_weno_field_flux(_f64(f), _f64(u), float(alpha), eps)


def weno_field_flux_z(f, u, alpha, eps=1e-6):
    """eq. (1) for one field with the WENO-Z weights (ablation)."""
    return lib().orc_weno_field_flux_z(_f64(f), _f64(u), float(alpha), eps)


# ---- point functions ----
def prim_to_cons(W, gamma=5.0 / 3.0):
    U = np.zeros(8)
    lib().orc_prim_to_cons(_f64(W), gamma, U)
    return U


def cons_to_prim(U, gamma=5.0 / 3.0):
    W = np.zeros(8)
    lib().orc_cons_to_prim(_f64(U), gamma, W)
    return W


def flux(U, direction, gamma=5.0 / 3.0):
    F = np.zeros(8)
    lib().orc_flux(_f64(U), int(direction), gamma, F)
    return F


def wave_speeds(U, direction, gamma=5.0 / 3.0):
    cf, ca, cs = C.c_double(), C.c_double(), C.c_double()
    lib().orc_wave_speeds(_f64(U), int(direction), gamma, C.byref(cf), C.byref(ca), C.byref(cs))
    return cf.value, ca.value, cs.value


def eigensystem(Wn, gamma=5.0 / 3.0):
    """Sweep-frame eigen-system at primitive state Wn -> (lam[8], L[8,8], R[8,8])."""
    lam = np.zeros(8)
    L = np.zeros(64)
    R = np.zeros(64)
    lib().orc_eigensystem(_f64(Wn), gamma, lam, L, R)
    return lam, L.reshape(8, 8), R.reshape(8, 8)


def interface_flux(Us, gamma=5.0 / 3.0, eps=1e-6):
    F = np.zeros(8)
    lib().orc_interface_flux(_f64(np.asarray(Us).reshape(48)), gamma, eps, F)
    return F


def interface_flux_z(Us, gamma=5.0 / 3.0, eps=1e-6):
    """The characteristic flux with the WENO-Z weights (ablation)."""
    F = np.zeros(8)
    lib().orc_interface_flux_z(_f64(np.asarray(Us, dtype=np.float64).reshape(-1)), gamma, eps, F)
    return F


def interface_flux_ex(Us, gamma=5.0 / 3.0, eps=1e-6, common_alpha=False):
    """(flux, largest weight deviation from linear) at one interface."""
    F = np.zeros(8)
    dev = C.c_double()
    lib().orc_interface_flux_ex(_f64(np.asarray(Us).reshape(48)), gamma, eps, int(common_alpha), F,
                                C.byref(dev))
    return F, dev.value


def linear_flux(Us, gamma=5.0 / 3.0):
    F = np.zeros(8)
    lib().orc_linear_flux(_f64(np.asarray(Us).reshape(48)), gamma, F)
    return F


# ---- grid operations ----
def flux_excess(Us, gamma=5.0 / 3.0, eps=1e-6):
    """Training label of the learned router (not part of the paper): how far
    the characteristic WENO flux of Sec. 2.1 departs from the linear
    fifth-order component-wise flux at one interface, per component relative
    to a stencil scale, maximised over the components:

      r = max_c |Fhat_c - Flin_c| / (a S_c),  a = max_j (|v_n| + c_f),
      S = max rho (mass), max (|m|_1 + rho a) (momenta),
          max |B|_1 + sqrt(max rho) a (fields), max E (energy),
    maxima over the six stencil cells, |.|_1 the sum of absolute components.
    """
    Us = np.asarray(Us, dtype=np.float64)
    Ff = interface_flux(Us, gamma, eps)
    Fl = linear_flux(Us, gamma)
    a = 0.0
    for j in range(6):
        cf = wave_speeds(Us[j], 0, gamma)[0]
        a = max(a, abs(Us[j, 1]) / Us[j, 0] + cf)
    rho = Us[:, 0]
    sm = (np.abs(Us[:, 1:4]).sum(1) + rho * a).max()
    sb = np.abs(Us[:, 4:7]).sum(1).max() + np.sqrt(rho.max()) * a
    S = np.array([rho.max(), sm, sm, sm, np.inf, sb, sb, Us[:, 7].max()])
    return float((np.abs(Ff - Fl) / (a * S)).max())


def _state(grid: Grid, u):
    if u.shape != grid.shape or u.dtype != np.float64 or not u.flags.c_contiguous:
        raise ValueError(f"state must be C-contiguous float64 {grid.shape}, got {u.shape} {u.dtype}")
    return u


def fill_ghosts(grid: Grid, u):
    g = grid.c()
    lib().orc_fill_ghosts(C.byref(g), _state(grid, u).reshape(-1))
    return u


def rhs(grid: Grid, u):
    g = grid.c()
    out = np.zeros(grid.shape)
    rc = lib().orc_rhs(C.byref(g), _state(grid, u).reshape(-1), out.reshape(-1))
    if rc != 0:
        raise FloatingPointError("oracle rhs: non-physical state")
    return out


def rhs_nofill(grid: Grid, u):
    """L(U) with the ghost zones of u taken as given (no refill)."""
    g = grid.c()
    out = np.zeros(grid.shape)
    rc = lib().orc_rhs_nofill(C.byref(g), _state(grid, u).reshape(-1), out.reshape(-1))
    if rc != 0:
        raise FloatingPointError("oracle rhs: non-physical state")
    return out


def rhs_linear(grid: Grid, u):
    """L(U) with the linear component-wise flux at every interface."""
    g = grid.c()
    out = np.zeros(grid.shape)
    rc = lib().orc_rhs_linear(C.byref(g), _state(grid, u).reshape(-1), out.reshape(-1))
    if rc != 0:
        raise FloatingPointError("oracle rhs: non-physical state")
    return out


def cfl_dt(grid: Grid, u):
    g = grid.c()
    dt = lib().orc_cfl_dt(C.byref(g), _state(grid, u).reshape(-1))
    if dt <= 0:
        raise FloatingPointError("oracle cfl_dt: non-physical state")
    return dt


def rk4_step(grid: Grid, u, dt):
    g = grid.c()
    rc = lib().orc_rk4_step(C.byref(g), _state(grid, u).reshape(-1), float(dt))
    if rc != 0:
        raise FloatingPointError("oracle rk4_step: non-physical state")
    return u


def ssprk3_step(grid: Grid, u, dt):
    """SSP-RK3 (Shu & Osher 1988): an ablation of the classical RK4."""
    g = grid.c()
    rc = lib().orc_ssprk3_step(C.byref(g), _state(grid, u).reshape(-1), float(dt))
    if rc != 0:
        raise FloatingPointError("oracle ssprk3_step: non-physical state")
    return u


def lf_global(grid: Grid, u, d):
    """Global LF speeds (7 fields) of the d-sweep of a state with filled
    ghosts (ablation of the per-stencil speed)."""
    out = np.zeros(7)
    lib().orc_lf_global(C.byref(grid.c()), _state(grid, u).reshape(-1), int(d), out)
    return out


def interface_flux_alpha(Us, alpha, gamma=5.0 / 3.0, eps=1e-6, z=0):
    """The characteristic flux of a 6x8 sweep-frame stencil with given LF
    speeds per field (ablation)."""
    F = np.zeros(8)
    lib().orc_interface_flux_alpha(_f64(Us).reshape(-1), gamma, eps, int(z), _f64(alpha), F)
    return F


def sums(grid: Grid, u):
    g = grid.c()
    out = np.zeros(8)
    lib().orc_sums(C.byref(g), _state(grid, u).reshape(-1), out)
    return out


def divb(grid: Grid, u):
    g = grid.c()
    mx, l1 = C.c_double(), C.c_double()
    lib().orc_divb(C.byref(g), _state(grid, u).reshape(-1), C.byref(mx), C.byref(l1))
    return mx.value, l1.value


def face_to_cell(grid: Grid, u):
    """Cell-centred state of a staggered (b_face) state, ghosts filled."""
    out = np.zeros(grid.shape)
    lib().orc_face_to_cell(C.byref(grid.c()), _state(grid, u).reshape(-1), out.reshape(-1))
    return out


def divb_face(grid: Grid, u):
    """Face divergence of a staggered (b_face) state: (max, mean) of |div b|."""
    mx, l1 = C.c_double(), C.c_double()
    lib().orc_divb_face(C.byref(grid.c()), _state(grid, u).reshape(-1), C.byref(mx), C.byref(l1))
    return mx.value, l1.value
