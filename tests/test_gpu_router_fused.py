"""The learned route on boxes whose x rows take the fused x sweep (rows of at
least 86 faces): the routed x tiles also apply the rho, m, E part of the RK
stage to every cell whose two x faces lie in the tile and are both smooth,
and a fix-up pass takes the cells next to troubled faces and those whose two
faces straddle consecutive tiles.  Checked against the plain fused FP32 path
(every interface troubled), the all-linear mode and the oracle's linear
right-hand side (every interface smooth), and for a mixed routing: cell by
cell where a cell's neighbourhood is routed one way, every hydro value
written, the telescoping sum of each hydro right-hand side, and the stage
form (each cell's accumulator advanced exactly once)."""
import math

import numpy as np
import pytest

from gpu_helpers import say, scaled_rhs_error
from oracle import oracle as O
from paper_1808_10633_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1808_10633_amd import router as R  # noqa: E402
from paper_1808_10633_amd import wombat as W  # noqa: E402

NX, NY, NZ = 96, 24, 20          # 97 x faces per row: the fused x sweep
H = 1.0 / NX
HYDRO = [0, 1, 2, 3, 7]


def _ctx(theta=None, mode=0, thr=0.5):
    ctx = W.Context(NX, NY, NZ, dx=H, dy=H, dz=H, precision=W.WW_FP32_MIXED, learned=1)
    if theta is not None:
        ctx.set_router(theta, thr, mode)
    return ctx


def _rhs(ctx, ug):
    d = torch.full_like(ug, float("nan"))
    ctx.rhs(ug, d)
    torch.cuda.synchronize()
    return d


def _state(seed, uniform_half=False):
    u = I.turbulence((NX, NY, NZ), mach=2.0, beta=5.0, seed=seed, kmax=6, dx=H).numpy().copy()
    if uniform_half:
        sl = (slice(None), slice(3, NZ + 3), slice(3, NY + 3), slice(3, 3 + NX // 2))
        u[sl] = u[sl].mean(axis=(1, 2, 3))[:, None, None, None]
    return u


def test_fused_routed_sweep_forced_and_extreme_routes():
    say(f"[learned fused x] {NX}x{NY}x{NZ}: all troubled vs plain, all smooth vs all-linear and the oracle")
    u = _state(71)
    ug = torch.from_numpy(u).cuda().float()
    sl = I.interior_slices(NX, NY, NZ)
    plain = _rhs(W.Context(NX, NY, NZ, dx=H, dy=H, dz=H, precision=W.WW_FP32_MIXED), ug)
    theta = R.init_params(11)
    hi = theta.clone()
    hi[-1] = 1e4
    ctx = _ctx(hi, 0)
    r1 = _rhs(ctx, ug)
    assert ctx.router_stats()[0] == 0
    assert torch.isfinite(r1[sl]).all()
    g = O.Grid(NX, NY, NZ, H, H, H)
    e1, _ = scaled_rhs_error(g.interior(r1.double().cpu().numpy()), g.interior(plain.double().cpu().numpy()),
                             g.interior(u), H)
    say(f"  all troubled (queued full WENO, every cell by the fix-up pass) vs plain fused FP32: {e1:.2e}")
    assert e1 < 1e-6
    lo = theta.clone()
    lo[-1] = -1e4
    ctx = _ctx(lo, 0)
    r0 = _rhs(ctx, ug)
    sm, tot, _ = ctx.router_stats()
    lin = _rhs(_ctx(lo, -1), ug)
    assert sm == tot and torch.equal(r0[sl], lin[sl])
    ref = O.rhs_linear(g, u)
    err, _ = scaled_rhs_error(g.interior(r0.double().cpu().numpy()), g.interior(ref), g.interior(u), H)
    say(f"  all smooth (in-tile tails + tile-boundary cells) vs the oracle's linear rhs: {err:.2e}")
    assert err < 2e-6


def test_fused_routed_sweep_mixed_routing():
    u = _state(72, uniform_half=True)
    ug = torch.from_numpy(u).cuda().float()
    sl = I.interior_slices(NX, NY, NZ)
    theta = R.init_params(7)
    plain = _rhs(W.Context(NX, NY, NZ, dx=H, dy=H, dz=H, precision=W.WW_FP32_MIXED), ug)
    lin = _rhs(_ctx(theta, -1), ug)
    ctx = _ctx()
    dims = (NX, NY, NZ)
    faces = []
    for d in range(3):
        lim = [dims[a] + (d == a) for a in range(3)]
        gr = torch.stack(torch.meshgrid(*[torch.arange(m) for m in lim], indexing="ij"), -1).reshape(-1, 3)
        faces.append(torch.cat([torch.full((len(gr), 1), d), gr], 1))
    where = torch.cat(faces).to(torch.int32).cuda().contiguous()
    X, _, _ = ctx.router_sample(ug, where)
    z = W.mlp_forward(theta, X).cpu()
    wh = where.cpu().long()
    inner = (wh[:, 1] >= 3) & (wh[:, 1] <= NX // 2 - 3)
    z0 = float(z[inner].max())
    tl = float(z[~inner].median())
    if abs(tl - z0) < 0.01:
        tl = z0 + 0.02
    ctx.set_router(theta, 1.0 / (1.0 + math.exp(-tl)), 0)
    mix = _rhs(ctx, ug)
    sm, tot, _ = ctx.router_stats()
    say(f"[learned fused x] mixed routing: {sm}/{tot} smooth")
    assert 0 < sm < tot
    # the queue order depends on the atomics; the result does not
    assert torch.equal(_rhs(ctx, ug)[sl], mix[sl])
    # every cell's hydro values written once the fix-up pass has run
    assert torch.isfinite(mix[sl]).all()
    # telescoping: each hydro rhs sums to round-off over the periodic box
    tel = max(abs(float(mix[sl][v].double().sum())) / float(mix[sl][v].double().abs().sum()) for v in HYDRO)
    say(f"  largest |sum of a hydro rhs| / sum of its |values|: {tel:.2e}")
    assert tel <= 2e-6
    # cells whose neighbourhood is routed one way equal that route
    per = torch.tensor(dims)
    anyt = torch.zeros(dims, dtype=torch.bool)
    anys = torch.zeros(dims, dtype=torch.bool)
    for flag, grid in ((z > tl - 1e-4, anyt), (z < tl + 1e-4, anys)):
        sel = wh[flag]
        c = sel[:, 1:] % per
        grid[c[:, 0], c[:, 1], c[:, 2]] = True
        c2 = sel[:, 1:].clone()
        c2[torch.arange(len(c2)), sel[:, 0]] -= 1
        c2 %= per
        grid[c2[:, 0], c2[:, 1], c2[:, 2]] = True

    def pool(gm):
        gp = torch.nn.functional.pad(gm[None, None].float(), (1, 1, 1, 1, 1, 1), mode="circular")
        return torch.nn.functional.max_pool3d(gp, 3, 1, 0)[0, 0] > 0
    fo = (~pool(anys)).permute(2, 1, 0)
    lo_ = (~pool(anyt)).permute(2, 1, 0)
    m, p_, l_ = mix[sl].cpu(), plain[sl].cpu(), lin[sl].cpu()
    say(f"  cells routed all-full {int(fo.sum())}, all-linear {int(lo_.sum())}")
    assert int(lo_.sum()) > 0 and int(fo.sum()) > 0
    assert torch.equal(m[:, lo_], l_[:, lo_])
    scale = p_.abs().amax(dim=(1, 2, 3), keepdim=True)[:, :, 0, 0]
    d = ((m[:, fo] - p_[:, fo]).abs() / scale).max()
    say(f"  full-only cells vs plain: {float(d):.2e} of each variable's largest |rhs|")
    assert float(d) < 1e-5
    # stage form (stage 2 of RK4: acc += dt/3 L in place): every cell once
    dt = 1e-4
    acc = torch.zeros_like(ug)
    out = torch.zeros_like(ug)
    ctx.stage(1, dt, ug, ug.clone(), acc, out)
    torch.cuda.synchronize()
    want = (dt / 3.0) * mix[sl].double()
    got = acc[sl].double()
    rel = ((got - want).abs().amax(dim=(1, 2, 3)) / want.abs().amax(dim=(1, 2, 3)).clamp_min(1e-30)).max()
    say(f"  stage accumulator vs dt/3 L: {float(rel):.2e}")
    assert float(rel) < 1e-5


def test_fused_routed_steps_match_their_routes():
    # whole RK4 steps (decisions of the first stage reused in stages 2-4):
    # every interface troubled equals the plain fused FP32 step up to FMA
    # contraction, every interface smooth equals the all-linear step bitwise
    say(f"[learned fused x] {NX}x{NY}x{NZ}: two RK4 steps per route")
    u = torch.from_numpy(_state(73)).cuda().float().contiguous()
    plain = W.Context(NX, NY, NZ, dx=H, dy=H, dz=H, precision=W.WW_FP32_MIXED)
    dt = plain.cfl_dt(u)
    up = u.clone()
    for _ in range(2):
        plain.step(up, dt)
    theta = R.init_params(13)
    hi = theta.clone()
    hi[-1] = 1e4
    ctx = _ctx(hi, 0)
    ut = u.clone()
    for _ in range(2):
        ctx.step(ut, dt)
    torch.cuda.synchronize()
    sl = I.interior_slices(NX, NY, NZ)
    S = up[sl].abs().amax(dim=(1, 2, 3)).double()
    e = float(((ut[sl] - up[sl]).abs().amax(dim=(1, 2, 3)).double() / S).max())
    say(f"  all troubled vs plain: {e:.2e}")
    assert e < 1e-6 and ctx.router_stats()[2] == 0
    lo = theta.clone()
    lo[-1] = -1e4
    ctx.set_router(lo, 0.5, -1)
    ul = u.clone()
    for _ in range(2):
        ctx.step(ul, dt)
    ctx.set_router(lo, 0.5, 0)
    ur = u.clone()
    for _ in range(2):
        ctx.step(ur, dt)
    torch.cuda.synchronize()
    assert ctx.router_stats()[2] == 0 and torch.equal(ur, ul)
