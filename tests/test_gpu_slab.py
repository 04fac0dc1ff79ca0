"""Slab mode (cfg.slab_planes): the RK4 stages run in z-slabs with the face
fluxes of one slab, the stage state updated in place through a three-plane
delay buffer, and two work arrays instead of three.  Every face flux and cell
update comes from the same kernels as the whole-box stage, so steps, stages
and right-hand sides equal the whole-box ones bit for bit: full slabs, a
ragged last slab, the smallest slab (3 planes), one slab covering the box,
FP64 and FP32, a 2-D x-z box with outflow faces."""
import numpy as np
import pytest

from gpu_helpers import say
from paper_1808_10633_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1808_10633_amd import wombat as W  # noqa: E402


def _steps(n, u0, nsteps, precision, **kw):
    ctx = W.Context(*n, precision=precision, **kw)
    u = u0.clone()
    dts = [ctx.step(u, 0.0) for _ in range(nsteps)]
    torch.cuda.synchronize()
    ctx.close()
    return u, dts


@pytest.mark.parametrize("slab", [8, 13, 3, 64])
def test_slab_steps_equal_whole_box_fp64(slab):
    n = (64, 64, 64)
    say(f"[slab] 64^3 FP64, 3 steps, slab_planes {slab}")
    u0 = I.turbulence(n, mach=1.0, beta=10.0, seed=81, device="cuda")
    ref, dref = _steps(n, u0, 3, W.WW_FP64)
    got, dgot = _steps(n, u0, 3, W.WW_FP64, slab_planes=slab)
    sl = I.interior_slices(*n)
    assert dref == dgot
    assert torch.equal(ref[sl], got[sl])


def test_slab_steps_equal_whole_box_fp32_and_2d_outflow():
    n = (48, 40, 36)
    say("[slab] 48x40x36 FP32, 3 steps, slab_planes 7")
    u0 = I.turbulence(n, mach=2.0, beta=1.0, seed=82, device="cuda").float().contiguous()
    ref, _ = _steps(n, u0, 3, W.WW_FP32_MIXED)
    got, _ = _steps(n, u0, 3, W.WW_FP32_MIXED, slab_planes=7)
    sl = I.interior_slices(*n)
    assert torch.equal(ref[sl], got[sl])
    n2 = (40, 1, 30)
    say("[slab] 40x1x30 FP64 outflow in x and z, 3 steps, slab_planes 4")
    u2 = I.turbulence(n2, mach=1.0, beta=3.0, seed=83, kmax=6, device="cuda")
    kw = dict(bc=(1, 1, 0, 0, 1, 1), dy=1.0)
    ref2, _ = _steps(n2, u2, 3, W.WW_FP64, **kw)
    got2, _ = _steps(n2, u2, 3, W.WW_FP64, slab_planes=4, **kw)
    sl2 = I.interior_slices(*n2)
    assert torch.equal(ref2[sl2], got2[sl2])


def test_fused_x_sweep_equals_separate_update():
    # rows of >= 86 faces take the x sweep with the rho, m, E update fused in
    # (the whole-box path); slab mode keeps the separate update: bit for bit
    n = (100, 24, 30)
    say("[slab] 100x24x30 FP64 and FP32, 3 steps: fused x sweep vs slabs of 8 (separate update)")
    for prec, dt_ in ((W.WW_FP64, torch.float64), (W.WW_FP32_MIXED, torch.float32)):
        u0 = I.turbulence(n, mach=1.5, beta=3.0, seed=85, kmax=6, dx=0.01, device="cuda").to(dt_).contiguous()
        kw = dict(dx=0.01, dy=0.01, dz=0.01)
        ref, dref = _steps(n, u0, 3, prec, **kw)
        got, dgot = _steps(n, u0, 3, prec, slab_planes=8, **kw)
        sl = I.interior_slices(*n)
        assert dref == dgot
        assert torch.equal(ref[sl], got[sl])


def test_slab_rhs_and_in_place_stage():
    n = (32, 24, 40)
    say("[slab] 32x24x40 FP64: rhs, and stage 1 written over its input")
    u = I.turbulence(n, mach=1.0, beta=10.0, seed=84, device="cuda")
    plain = W.Context(*n, precision=W.WW_FP64)
    slab = W.Context(*n, precision=W.WW_FP64, slab_planes=6)
    d1, d2 = torch.zeros_like(u), torch.zeros_like(u)
    plain.rhs(u.clone(), d1)
    slab.rhs(u.clone(), d2)
    sl = I.interior_slices(*n)
    assert torch.equal(d1[sl], d2[sl])
    dt = plain.cfl_dt(u)
    # stage 1 of a step: u0 = u, us = U_2 (from stage 0), acc
    us = u.clone()
    acc_a, out_a = torch.zeros_like(u), torch.zeros_like(u)
    plain.stage(0, dt, u, u.clone(), acc_a, us)
    acc_b = acc_a.clone()
    plain.stage(1, dt, u, us.clone(), acc_a, out_a)
    inplace = us.clone()
    slab.stage(1, dt, u, inplace, acc_b, inplace)
    torch.cuda.synchronize()
    assert torch.equal(out_a[sl], inplace[sl])
    assert torch.equal(acc_a[sl], acc_b[sl])
    # the plain context still refuses the alias
    with pytest.raises(W.WenoError, match="alias"):
        plain.stage(1, dt, u, inplace, acc_b, inplace)
    plain.close()
    slab.close()


def test_slab_mode_uses_less_memory():
    n = (96, 96, 96)
    free0 = torch.cuda.mem_get_info()[0]
    a = W.Context(*n, precision=W.WW_FP64)
    torch.cuda.synchronize()
    used_plain = free0 - torch.cuda.mem_get_info()[0]
    a.close()
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    b = W.Context(*n, precision=W.WW_FP64, slab_planes=8)
    torch.cuda.synchronize()
    used_slab = free1 - torch.cuda.mem_get_info()[0]
    b.close()
    state = 8 * 102 ** 3 * 8
    say(f"[slab] 96^3 FP64 context: {used_plain / 1e6:.0f} MB whole box, {used_slab / 1e6:.0f} MB slabs of 8")
    assert used_slab < used_plain - state
