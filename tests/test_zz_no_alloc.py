"""wombat_weno_rhs_noalloc, the right-hand side for callers that cannot
allocate, against wombat_weno_rhs through the C ABI: bit for bit on two calls
in a row (a 64^3 FP64 box, then a smaller 2-D FP32 box with outflow faces),
no allocation by the library across the calls, and a box beyond the fixed
scratch refused with a clear error.  (Named to be collected last.)"""
import ctypes as C

import numpy as np
import pytest

from gpu_helpers import say
from paper_1808_10633_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1808_10633_amd import wombat as W  # noqa: E402


def _noalloc(cfg, u, dudt):
    # the C ABI call itself (the binding's rhs_noalloc raises instead)
    return W.lib().wombat_weno_rhs_noalloc(C.byref(cfg), C.c_void_p(u.data_ptr()), C.c_void_p(dudt.data_ptr()))


def _case(n, precision, seed, bc=(0, 0, 0, 0, 0, 0)):
    nx, ny, nz = n
    dt = torch.float64 if precision == W.WW_FP64 else torch.float32
    u = I.turbulence(n, mach=1.5, beta=3.0, seed=seed, kmax=min(6.0, min(v for v in n if v > 1) / 2 - 1),
                     device="cuda").to(dt).contiguous()
    ctx = W.Context(nx, ny, nz, precision=precision, bc=bc)
    ref = torch.zeros_like(u)
    ctx.rhs(u, ref)
    torch.cuda.synchronize()
    return ctx, u, ref


def test_rhs_noalloc_matches_rhs_twice():
    torch.cuda.set_device(0)
    cases = [((64, 64, 64), W.WW_FP64, 71, (0, 0, 0, 0, 0, 0)),
             ((40, 27, 1), W.WW_FP32_MIXED, 72, (1, 1, 0, 0, 0, 0))]
    for n, prec, seed, bc in cases:
        say(f"[noalloc] case {n} precision {prec}")
        ctx, u, ref = _case(n, prec, seed, bc)
        before = W.alloc_count()
        got = torch.full_like(u, float("nan"))
        rc = _noalloc(ctx.cfg, u, got)
        assert rc == W.WW_OK, W.last_error()
        torch.cuda.synchronize()
        assert W.alloc_count() == before
        sl = (slice(None),) + tuple(slice(3, 3 + v) if v > 1 else slice(0, 1) for v in (n[2], n[1], n[0]))
        a = got[sl].cpu().numpy()
        b = ref[sl].cpu().numpy()
        say(f"  max |noalloc - rhs| = {np.abs(a - b).max():.3e}")
        assert np.array_equal(a, b)
        ctx.close()


def test_rhs_noalloc_refuses_a_box_beyond_its_scratch():
    cfg = W.make_config(256, 256, 256, stream=torch.cuda.current_stream().cuda_stream)
    u = torch.zeros(8, dtype=torch.float64, device="cuda")
    rc = _noalloc(cfg, u, torch.zeros_like(u))
    assert rc == W.WW_ERR_INVALID_ARG
    assert "too large" in W.last_error()
