"""Thin ctypes binding of the C ABI in ``include/wombat_weno.h``.

Argument marshalling only: every step of the stage runs in the HIP library
``libwombat_weno.so``.  Device memory and streams come from PyTorch; tensors
are passed by ``data_ptr()``.  There is no fallback: without the built
library (or without a GPU) every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwombat_weno.so")

WW_OK = 0
WW_ERR_INVALID_ARG = -1
WW_ERR_UNSUPPORTED = -2
WW_ERR_OOM = -3
WW_ERR_HIP = -4
WW_ERR_NONPHYSICAL = -5
WW_ERR_USER_BC = -6
WW_ERR_STATE = -7
_NAMES = {0: "WW_OK", -1: "WW_ERR_INVALID_ARG", -2: "WW_ERR_UNSUPPORTED", -3: "WW_ERR_OOM",
          -4: "WW_ERR_HIP", -5: "WW_ERR_NONPHYSICAL", -6: "WW_ERR_USER_BC", -7: "WW_ERR_STATE"}

ABI_VERSION = 6          # layout of Config below
WW_FP64 = 0
WW_FP32_MIXED = 1
WEIGHTS_JS, WEIGHTS_Z = 0, 1
RK4, SSPRK3 = 0, 1
LF_LOCAL, LF_GLOBAL = 0, 1
BC_PERIODIC, BC_OUTFLOW, BC_USER = 0, 1, 2
B_CELL, B_FACE = 0, 1

USER_BC_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p)


class Config(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("ng", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("gamma", C.c_double), ("cfl", C.c_double), ("eps", C.c_double),
                ("precision", C.c_int), ("bc", C.c_int * 6),
                ("user_bc", USER_BC_FN), ("user_bc_ctx", C.c_void_p),
                ("stream", C.c_void_p), ("device", C.c_int), ("weights", C.c_int),
                ("integrator", C.c_int), ("lf_speed", C.c_int), ("learned", C.c_int),
                ("slab_planes", C.c_int), ("b_storage", C.c_int)]


class WenoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1808_10633_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, d = C.c_void_p, C.c_int, C.c_double
        L.wombat_weno_abi_version.restype = i32
        if L.wombat_weno_abi_version() != ABI_VERSION:
            raise RuntimeError(f"{LIB_PATH} has ABI {L.wombat_weno_abi_version()}, the binding "
                               f"expects {ABI_VERSION}: rebuild it")
        L.wombat_weno_config_default.argtypes = [C.POINTER(Config)]
        L.wombat_weno_validate_config.argtypes = [C.POINTER(Config)]
        L.wombat_weno_state_elems.argtypes = [C.POINTER(Config)]
        L.wombat_weno_state_elems.restype = C.c_int64
        L.wombat_weno_init.argtypes = [C.POINTER(Config), C.POINTER(vp)]
        L.wombat_weno_destroy.argtypes = [vp]
        L.wombat_weno_destroy.restype = None
        L.wombat_weno_last_error.argtypes = [vp]
        L.wombat_weno_last_error.restype = C.c_char_p
        L.wombat_weno_fill_ghosts.argtypes = [vp, vp]
        L.wombat_weno_cfl_dt.argtypes = [vp, vp, C.POINTER(d)]
        L.wombat_weno_cfl_dt_device.argtypes = [vp, vp, vp, vp]
        L.wombat_weno_rhs.argtypes = [vp, vp, vp]
        L.wombat_weno_stage.argtypes = [vp, i32, d, vp, vp, vp, vp]
        L.wombat_weno_step.argtypes = [vp, vp, d, C.POINTER(d)]
        L.wombat_weno_sums.argtypes = [vp, vp, C.POINTER(d)]
        L.wombat_weno_divb.argtypes = [vp, vp, C.POINTER(d), C.POINTER(d)]
        L.wombat_weno_time_kernels.argtypes = [vp, vp, i32, C.POINTER(d)]
        L.wombat_weno_alloc_count.restype = C.c_int64
        L.wombat_weno_rhs_noalloc.argtypes = [C.POINTER(Config), vp, vp]
        L.wombat_weno_batch_init.argtypes = [C.POINTER(Config), i32, C.POINTER(C.c_int32), C.POINTER(vp)]
        L.wombat_weno_batch_destroy.argtypes = [vp]
        L.wombat_weno_batch_destroy.restype = None
        L.wombat_weno_batch_last_error.argtypes = [vp]
        L.wombat_weno_batch_last_error.restype = C.c_char_p
        L.wombat_weno_batch_arena_elems.argtypes = [vp]
        L.wombat_weno_batch_arena_elems.restype = C.c_int64
        L.wombat_weno_batch_patch_offset.argtypes = [vp, i32]
        L.wombat_weno_batch_patch_offset.restype = C.c_int64
        L.wombat_weno_batch_step.argtypes = [vp, vp]
        L.wombat_weno_batch_graph_steps.argtypes = [vp, vp, i32]
        L.wombat_weno_batch_dt.argtypes = [vp, vp, vp]
        L.wombat_weno_batch_shape.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
        L.wombat_weno_batch_autotune.argtypes = [vp, vp, C.c_char_p, C.POINTER(d)]
        L.wombat_weno_set_router.argtypes = [vp, vp, d, i32]
        L.wombat_weno_router_stats.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                               C.POINTER(C.c_int64)]
        L.wombat_weno_router_sample.argtypes = [vp, vp, vp, i32, vp, vp, vp]
        L.wombat_mlp_param_count.restype = i32
        L.wombat_mlp_forward.argtypes = [vp, vp, vp, i32, vp]
        L.wombat_mlp_grad_workspace.argtypes = [i32]
        L.wombat_mlp_grad_workspace.restype = C.c_int64
        L.wombat_mlp_grad.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp]
        L.wombat_mlp_adam.argtypes = [vp, vp, vp, vp, vp, i32, C.c_float, C.c_float, C.c_float, C.c_float]
        _lib = L
    return _lib


def alloc_count() -> int:
    """Device and pinned-host allocations the library has made so far."""
    return int(lib().wombat_weno_alloc_count())


def rhs_noalloc(cfg, u, dudt):
    """wombat_weno_rhs_noalloc: L(u) into dudt for the configuration cfg
    (a Config), without a context and without allocation."""
    _check(lib().wombat_weno_rhs_noalloc(C.byref(cfg), C.c_void_p(u.data_ptr()), C.c_void_p(dudt.data_ptr())))


def last_error(ctx=None) -> str:
    s = lib().wombat_weno_last_error(ctx)
    return s.decode() if s else ""


def make_config(nx, ny=1, nz=1, *, dx=None, dy=None, dz=None, gamma=5.0 / 3.0, cfl=0.4,
                eps=1e-6, precision=WW_FP64, bc=(0, 0, 0, 0, 0, 0), user_bc=None,
                stream=None, device=0, weights=WEIGHTS_JS, integrator=RK4,
                lf_speed=LF_LOCAL, learned=0, slab_planes=0, b_storage=B_CELL) -> Config:
    cfg = Config()
    lib().wombat_weno_config_default(C.byref(cfg))
    cfg.nx, cfg.ny, cfg.nz, cfg.ng = nx, ny, nz, 3
    cfg.dx = 1.0 / nx if dx is None else dx
    cfg.dy = (1.0 / ny if ny > 1 else 1.0) if dy is None else dy
    cfg.dz = (1.0 / nz if nz > 1 else 1.0) if dz is None else dz
    cfg.gamma, cfg.cfl, cfg.eps, cfg.precision = gamma, cfl, eps, precision
    for i in range(6):
        cfg.bc[i] = int(bc[i])
    if user_bc is not None:
        cfg.user_bc = user_bc
    cfg.stream = stream
    cfg.device = device
    cfg.weights = weights
    cfg.integrator = integrator
    cfg.lf_speed = lf_speed
    cfg.learned = int(learned)
    cfg.slab_planes = int(slab_planes)
    cfg.b_storage = int(b_storage)
    return cfg


def _check(code, ctx=None):
    if code != WW_OK:
        raise WenoError(code, last_error(ctx))


class Context:
    """One solver context (a ``wombat_weno_t``) for a fixed box.

    ``state`` tensors must be contiguous CUDA tensors of shape
    (8, nz+2gz, ny+2gy, nx+2gx) and dtype float64 (WW_FP64) or float32
    (WW_FP32_MIXED), on the context's device.
    """

    def __init__(self, nx, ny=1, nz=1, **kw):
        import torch
        if "stream" not in kw or kw["stream"] is None:
            kw["stream"] = torch.cuda.current_stream().cuda_stream
        if "device" not in kw:
            kw["device"] = torch.cuda.current_device()
        self.cfg = make_config(nx, ny, nz, **kw)
        self._user_bc = kw.get("user_bc")
        h = C.c_void_p()
        _check(lib().wombat_weno_init(C.byref(self.cfg), C.byref(h)))
        self.h = h
        self.dtype = torch.float64 if self.cfg.precision == WW_FP64 else torch.float32
        g = [3 if n > 1 else 0 for n in (nx, ny, nz)]
        self.shape = (8, nz + 2 * g[2], ny + 2 * g[1], nx + 2 * g[0])

    def close(self):
        if getattr(self, "h", None):
            lib().wombat_weno_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ptr(self, t, name):
        if t is None:
            return None
        if (not t.is_cuda or t.dtype != self.dtype or tuple(t.shape) != self.shape
                or not t.is_contiguous()):
            raise ValueError(f"{name}: need contiguous cuda {self.dtype} {self.shape}, got "
                             f"{t.device} {t.dtype} {tuple(t.shape)}")
        return C.c_void_p(t.data_ptr())

    def new_state(self):
        import torch
        return torch.zeros(self.shape, dtype=self.dtype, device=f"cuda:{self.cfg.device}")

    def fill_ghosts(self, u):
        _check(lib().wombat_weno_fill_ghosts(self.h, self._ptr(u, "u")), self.h)

    def cfl_dt(self, u) -> float:
        dt = C.c_double()
        _check(lib().wombat_weno_cfl_dt(self.h, self._ptr(u, "u"), C.byref(dt)), self.h)
        return dt.value

    def cfl_dt_device(self, u, d_dt, d_flag):
        _check(lib().wombat_weno_cfl_dt_device(self.h, self._ptr(u, "u"), C.c_void_p(d_dt.data_ptr()),
                                               C.c_void_p(d_flag.data_ptr())), self.h)

    def rhs(self, u, dudt):
        _check(lib().wombat_weno_rhs(self.h, self._ptr(u, "u"), self._ptr(dudt, "dudt")), self.h)

    def stage(self, s, dt, u0, us_in, acc, us_out):
        _check(lib().wombat_weno_stage(self.h, int(s), float(dt), self._ptr(u0, "u0"),
                                       self._ptr(us_in, "us_in"), self._ptr(acc, "acc"),
                                       self._ptr(us_out, "us_out")), self.h)

    def step(self, u, dt=0.0) -> float:
        used = C.c_double()
        _check(lib().wombat_weno_step(self.h, self._ptr(u, "u"), float(dt), C.byref(used)), self.h)
        return used.value

    def sums(self, u):
        out = (C.c_double * 8)()
        _check(lib().wombat_weno_sums(self.h, self._ptr(u, "u"), out), self.h)
        return list(out)

    KERNELS = ("ghosts", "sweep_x", "sweep_y", "sweep_z", "update_stage", "cfl", "update_rhs")

    def time_kernels(self, u, reps=10):
        """Average ms per launch, in the order of KERNELS: ghosts, sweeps x, y,
        z, the update in the stage forms of a step (their mean), the CFL
        reduction, the update writing L(U) only."""
        out = (C.c_double * 7)()
        _check(lib().wombat_weno_time_kernels(self.h, self._ptr(u, "u"), int(reps), out), self.h)
        return list(out)

    def set_router(self, theta, threshold=0.5, mode=0):
        """Learned routing of the sweeps (FP32 contexts); theta=None switches it off."""
        self._theta = theta
        ptr = None if theta is None else C.c_void_p(theta.data_ptr())
        _check(lib().wombat_weno_set_router(self.h, ptr, float(threshold), int(mode)), self.h)

    def router_stats(self):
        """(interfaces routed smooth in the last rhs/stage, interfaces swept,
        routed steps redone with full WENO since init)."""
        s, t, f = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().wombat_weno_router_stats(self.h, C.byref(s), C.byref(t), C.byref(f)), self.h)
        return s.value, t.value, f.value

    def router_sample(self, u, where):
        """where: int32 cuda tensor (n, 4) of (dir, i, j, k) ->
        (X (n, 48), weight deviation (n,), flux excess (n,))."""
        import torch
        n = where.shape[0]
        if where.dtype != torch.int32 or not where.is_contiguous() or tuple(where.shape[1:]) != (4,):
            raise ValueError("where must be a contiguous int32 tensor of shape (n, 4)")
        X = torch.empty((n, 48), dtype=torch.float32, device=u.device)
        dev = torch.empty(n, dtype=torch.float32, device=u.device)
        ex = torch.empty(n, dtype=torch.float32, device=u.device)
        _check(lib().wombat_weno_router_sample(self.h, self._ptr(u, "u"), C.c_void_p(where.data_ptr()), n,
                                               C.c_void_p(X.data_ptr()), C.c_void_p(dev.data_ptr()),
                                               C.c_void_p(ex.data_ptr())), self.h)
        return X, dev, ex

    def divb(self, u):
        mx, l1 = C.c_double(), C.c_double()
        _check(lib().wombat_weno_divb(self.h, self._ptr(u, "u"), C.byref(mx), C.byref(l1)), self.h)
        return mx.value, l1.value


class Batch:
    """Many independent periodic patches in one arena (``wombat_weno_batch_t``).

    ``dims``: sequence of (nx, ny, nz) per patch.  The arena is a 1-D contiguous
    CUDA tensor of ``arena_elems`` elements; ``view(arena, p)`` gives patch p's
    padded state (8, nz+6, ny+6, nx+6).
    """

    def __init__(self, dims, dx, precision=WW_FP32_MIXED, gamma=5.0 / 3.0, cfl=0.4, eps=1e-6,
                 stream=None, device=None):
        import numpy as np
        import torch
        self.dims = [tuple(int(v) for v in d) for d in dims]
        cfg = make_config(8, 8, 8, dx=dx, dy=dx, dz=dx, gamma=gamma, cfl=cfl, eps=eps,
                          precision=precision,
                          stream=torch.cuda.current_stream().cuda_stream if stream is None else stream,
                          device=torch.cuda.current_device() if device is None else device)
        self.cfg = cfg
        arr = np.ascontiguousarray(np.array(self.dims, dtype=np.int32).reshape(-1))
        h = C.c_void_p()
        rc = lib().wombat_weno_batch_init(C.byref(cfg), len(self.dims),
                                          arr.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(h))
        if rc != WW_OK:
            raise WenoError(rc, lib().wombat_weno_batch_last_error(None).decode())
        self.h = h
        self.dtype = torch.float64 if precision == WW_FP64 else torch.float32
        self.arena_elems = int(lib().wombat_weno_batch_arena_elems(h))
        self.offsets = [int(lib().wombat_weno_batch_patch_offset(h, p)) for p in range(len(self.dims))]

    def _check(self, rc):
        if rc != WW_OK:
            raise WenoError(rc, lib().wombat_weno_batch_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().wombat_weno_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_arena(self):
        import torch
        return torch.zeros(self.arena_elems, dtype=self.dtype, device=f"cuda:{self.cfg.device}")

    def view(self, arena, p):
        nx, ny, nz = self.dims[p]
        n = 8 * (nx + 6) * (ny + 6) * (nz + 6)
        o = self.offsets[p]
        return arena[o:o + n].view(8, nz + 6, ny + 6, nx + 6)

    def _ptr(self, arena):
        if (not arena.is_cuda or arena.dtype != self.dtype or arena.numel() != self.arena_elems
                or not arena.is_contiguous()):
            raise ValueError("arena: need a contiguous cuda tensor of arena_elems elements")
        return C.c_void_p(arena.data_ptr())

    def step(self, arena):
        self._check(lib().wombat_weno_batch_step(self.h, self._ptr(arena)))

    def graph_steps(self, arena, nsteps):
        self._check(lib().wombat_weno_batch_graph_steps(self.h, self._ptr(arena), int(nsteps)))

    def dt(self):
        import numpy as np
        d = np.zeros(len(self.dims))
        f = np.zeros(len(self.dims), dtype=np.int32)
        self._check(lib().wombat_weno_batch_dt(self.h, d.ctypes.data_as(C.c_void_p),
                                               f.ctypes.data_as(C.c_void_p)))
        return d, f

    def shape(self):
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        self._check(lib().wombat_weno_batch_shape(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def autotune(self, arena, cache_path=None):
        ms = C.c_double()
        self._check(lib().wombat_weno_batch_autotune(self.h, self._ptr(arena),
                                                     cache_path.encode() if cache_path else None,
                                                     C.byref(ms)))
        return ms.value


# ---- MLP of the learned router (stream = torch's current stream) ----

def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def mlp_param_count():
    return int(lib().wombat_mlp_param_count())


def mlp_forward(theta, X):
    import torch
    n = X.shape[0]
    out = torch.empty(n, dtype=torch.float32, device=X.device)
    _check(lib().wombat_mlp_forward(_stream(), C.c_void_p(theta.data_ptr()), C.c_void_p(X.data_ptr()), n,
                                    C.c_void_p(out.data_ptr())))
    return out


def mlp_grad(theta, X, t, work=None):
    import torch
    n = X.shape[0]
    if work is None:
        work = torch.empty(int(lib().wombat_mlp_grad_workspace(n)), dtype=torch.float32, device=X.device)
    g = torch.empty(mlp_param_count(), dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    _check(lib().wombat_mlp_grad(_stream(), C.c_void_p(theta.data_ptr()), C.c_void_p(X.data_ptr()),
                                 C.c_void_p(t.data_ptr()), n, C.c_void_p(work.data_ptr()),
                                 C.c_void_p(g.data_ptr()), C.c_void_p(loss.data_ptr())))
    return g, loss


def mlp_adam(theta, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(lib().wombat_mlp_adam(_stream(), C.c_void_p(theta.data_ptr()), C.c_void_p(m.data_ptr()),
                                 C.c_void_p(v.data_ptr()), C.c_void_p(grad.data_ptr()), int(step),
                                 float(lr), float(beta1), float(beta2), float(eps)))
