"""Batched form: many independent periodic patches of uneven sizes in one
arena, one persistent launch per RK stage, per-patch CFL time steps, HIP
graph replay, autotuned launch shape.

Each patch of a batched step must equal the single-box step of the same patch
with the same time step (same device functions; compared to 1e-13 of the
state scale, in practice bitwise), and the CPU oracle (<= 1e-11 scaled)."""
import os

import numpy as np
import pytest

from gpu_helpers import random_smooth, say, scaled_state_error
from oracle import oracle as O
from paper_1808_10633_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1808_10633_amd import wombat as W  # noqa: E402

DX = 1.0 / 64


def fill(batch, arena, seed0=4000, mach=(0.3, 2.0), beta=(1.0, 1e4)):
    rng = np.random.default_rng(seed0)
    for p, (nx, ny, nz) in enumerate(batch.dims):
        m = rng.uniform(*mach)
        b = 10 ** rng.uniform(np.log10(beta[0]), np.log10(beta[1]))
        u = I.turbulence((nx, ny, nz), mach=m, beta=b, seed=seed0 + p, dx=DX, device="cuda")
        batch.view(arena, p).copy_(u.to(batch.dtype))


DIMS = [(8, 12, 16), (16, 16, 16), (24, 8, 12), (12, 20, 9), (33, 10, 8), (9, 9, 70), (64, 8, 8)]


def test_batch_step_equals_single_box_steps():
    say("[batch] fp64 vs single-box steps")
    bt = W.Batch(DIMS, DX, precision=W.WW_FP64)
    ar = bt.new_arena()
    fill(bt, ar)
    before = [bt.view(ar, p).clone() for p in range(len(DIMS))]
    bt.step(ar)
    dts, flags = bt.dt()
    assert (flags == 0).all()
    worst = 0.0
    for p, (nx, ny, nz) in enumerate(DIMS):
        ctx = W.Context(nx, ny, nz, dx=DX, dy=DX, dz=DX, precision=W.WW_FP64)
        u = before[p].clone()
        assert abs(ctx.cfl_dt(u) - dts[p]) <= 1e-14 * dts[p]
        ctx.step(u, float(dts[p]))
        torch.cuda.synchronize()
        sl = I.interior_slices(nx, ny, nz)
        a = bt.view(ar, p)[sl].cpu().numpy()
        b = u[sl].cpu().numpy()
        err, _ = scaled_state_error(a, b)
        worst = max(worst, err)
    say(f"  worst scaled difference batch vs single-box {worst:.3e}")
    assert worst < 1e-13


@pytest.mark.parametrize("precision", [W.WW_FP64, W.WW_FP32_MIXED])
def test_small_patches_equal_single_box_steps(precision):
    # edges 4..7: flattened x rows of 4-7 cells (up to 53 rows per tile)
    dims = [(4, 4, 4), (5, 6, 7), (6, 4, 9), (7, 7, 4), (4, 9, 5)]
    say(f"[batch] small patches {dims}, precision {precision}")
    bt = W.Batch(dims, DX, precision=precision)
    ar = bt.new_arena()
    for p, (nx, ny, nz) in enumerate(dims):
        u = random_smooth(nx, ny, nz, seed=300 + p, amp=0.2)
        bt.view(ar, p).copy_(torch.from_numpy(u).to(bt.view(ar, p).dtype))
    before = [bt.view(ar, p).clone() for p in range(len(dims))]
    bt.step(ar)
    dts, flags = bt.dt()
    assert (flags == 0).all()
    worst = 0.0
    for p, (nx, ny, nz) in enumerate(dims):
        ctx = W.Context(nx, ny, nz, dx=DX, dy=DX, dz=DX, precision=precision)
        u = before[p].clone()
        ctx.step(u, float(dts[p]))
        torch.cuda.synchronize()
        sl = I.interior_slices(nx, ny, nz)
        err, _ = scaled_state_error(bt.view(ar, p)[sl].double().cpu().numpy(), u[sl].double().cpu().numpy())
        worst = max(worst, err)
    say(f"  worst scaled difference batch vs single-box {worst:.3e}")
    assert worst < (1e-13 if precision == W.WW_FP64 else 1e-6)


def test_batch_against_oracle():
    say("[batch] fp64 vs oracle")
    dims = [(8, 10, 12), (12, 8, 9)]
    bt = W.Batch(dims, DX, precision=W.WW_FP64)
    ar = bt.new_arena()
    fill(bt, ar, seed0=4100)
    refs = [bt.view(ar, p).cpu().numpy().copy() for p in range(len(dims))]
    bt.step(ar)
    dts, _ = bt.dt()
    for p, (nx, ny, nz) in enumerate(dims):
        g = O.Grid(nx, ny, nz, DX, DX, DX)
        dto = O.cfl_dt(g, refs[p])
        assert abs(dto - dts[p]) <= 1e-14 * dto
        O.rk4_step(g, refs[p], dto)
        err, _ = scaled_state_error(g.interior(bt.view(ar, p).cpu().numpy()), g.interior(refs[p]))
        say(f"  patch {p}: scaled error {err:.2e}")
        assert err < 1e-11


def test_batch_config4_patches_against_oracle():
    # 16 patches of the 4096-patch workload (edges drawn from {16, 24, 32, 48,
    # 64} per axis, rms Mach in [0.3, 2], beta in [1, 1e4], seed 4000 + p):
    # one step of the FP64 batched form against the oracle (<= 1e-11 scaled)
    # and of the FP32 form against the same oracle step (relative L1 and
    # Linf per variable, the precision form's error measure)
    rng = np.random.default_rng(4000)
    dims = [tuple(int(v) for v in rng.choice([16, 24, 32, 48, 64], size=3)) for _ in range(16)]
    say(f"[batch] 16 config-4 patches vs the oracle: {dims}")
    b64 = W.Batch(dims, DX, precision=W.WW_FP64)
    a64 = b64.new_arena()
    fill(b64, a64)
    refs = [b64.view(a64, p).cpu().numpy().copy() for p in range(len(dims))]
    b32 = W.Batch(dims, DX, precision=W.WW_FP32_MIXED)
    a32 = b32.new_arena()
    for p in range(len(dims)):
        b32.view(a32, p).copy_(b64.view(a64, p).float())
    b64.step(a64)
    b32.step(a32)
    dts, flags = b64.dt()
    dts32, _ = b32.dt()
    assert (flags == 0).all()
    O.set_threads(max(1, min(16, len(os.sched_getaffinity(0)))))
    worst64 = worst_l1 = worst_linf = 0.0
    try:
        for p, (nx, ny, nz) in enumerate(dims):
            g = O.Grid(nx, ny, nz, DX, DX, DX)
            dto = O.cfl_dt(g, refs[p])
            assert abs(dto - dts[p]) <= 1e-14 * dto
            assert abs(dts32[p] - dto) <= 1e-5 * dto
            O.rk4_step(g, refs[p], dto)
            ref = g.interior(refs[p])
            err, _ = scaled_state_error(g.interior(b64.view(a64, p).cpu().numpy()), ref)
            worst64 = max(worst64, err)
            got32 = g.interior(b32.view(a32, p).double().cpu().numpy())
            for v in range(8):
                r = np.abs(ref[v])
                if r.max() == 0:
                    continue
                d = np.abs(got32[v] - ref[v])
                worst_l1 = max(worst_l1, d.mean() / r.mean())
                worst_linf = max(worst_linf, d.max() / r.max())
    finally:
        O.set_threads(1)
    say(f"  FP64 worst scaled error {worst64:.2e}; FP32 worst relative L1 {worst_l1:.2e}, Linf {worst_linf:.2e}")
    assert worst64 < 1e-11
    assert worst_l1 < 1e-5 and worst_linf < 1e-3


def test_batch_graph_replays_match_eager():
    say("[batch] graph replays")
    rng = np.random.default_rng(9)
    dims = [tuple(int(v) for v in rng.choice([8, 12, 16, 24], size=3)) for _ in range(20)]
    bt = W.Batch(dims, DX, precision=W.WW_FP32_MIXED)
    ga = bt.new_arena()
    fill(bt, ga, seed0=4200)
    ea = ga.clone()
    for rep in range(3):
        bt.graph_steps(ga, 1)
        torch.cuda.synchronize()
        bt.step(ea)                   # eager work between the replays
        torch.cuda.synchronize()
        assert torch.equal(ga, ea), f"replay {rep} differs"
    bt.graph_steps(ga, 2)
    bt.step(ea)
    bt.step(ea)
    torch.cuda.synchronize()
    assert torch.equal(ga, ea)


def test_batch_autotune_and_cache(tmp_path):
    say("[batch] autotune")
    rng = np.random.default_rng(3)
    dims = [tuple(int(v) for v in rng.choice([16, 24, 32], size=3)) for _ in range(64)]
    bt = W.Batch(dims, DX, precision=W.WW_FP32_MIXED)
    ar = bt.new_arena()
    fill(bt, ar, seed0=4300)
    snap = ar.clone()
    cache = str(tmp_path / "tune.jsonl")
    ms = bt.autotune(ar, cache)
    ft, bpc, nb = bt.shape()
    say(f"  best {ms:.3f} ms/step ft={ft} blocks/CU={bpc} blocks={nb}")
    assert ms > 0 and ft in (4, 8, 12, 16) and 1 <= bpc <= 4
    assert torch.equal(ar, snap)          # the caller's arena is untouched
    assert os.path.exists(cache)
    bt2 = W.Batch(dims, DX, precision=W.WW_FP32_MIXED)
    assert bt2.autotune(ar, cache) == -1.0
    assert bt2.shape()[:2] == (ft, bpc)
    # stepping with the tuned shape gives the same result as the default shape
    bt3 = W.Batch(dims, DX, precision=W.WW_FP32_MIXED)
    a2, a3 = ar.clone(), ar.clone()
    bt2.step(a2)
    bt3.step(a3)
    torch.cuda.synchronize()
    assert torch.equal(a2, a3)


def test_batch_fp32_vs_fp64():
    say("[batch] fp32 vs fp64, 5 steps")
    rng = np.random.default_rng(4)
    dims = [tuple(int(v) for v in rng.choice([16, 24, 32], size=3)) for _ in range(12)]
    b64 = W.Batch(dims, DX, precision=W.WW_FP64)
    b32 = W.Batch(dims, DX, precision=W.WW_FP32_MIXED)
    a64 = b64.new_arena()
    fill(b64, a64, seed0=4400)
    a32 = a64.float().contiguous()
    for _ in range(5):
        b64.step(a64)
        b32.step(a32)
    torch.cuda.synchronize()
    worst = 0.0
    for p, (nx, ny, nz) in enumerate(dims):
        sl = I.interior_slices(nx, ny, nz)
        a = b32.view(a32, p)[sl].double()
        b = b64.view(a64, p)[sl]
        d = (a - b).abs().reshape(8, -1).mean(1) / b.abs().reshape(8, -1).mean(1).clamp_min(1e-300)
        worst = max(worst, float(d.max()))
    say(f"  worst per-variable relative L1 {worst:.2e}")
    assert worst < 1e-5


def test_batch_nonphysical_patch_is_flagged():
    dims = [(8, 8, 8), (12, 12, 12), (8, 12, 16)]
    bt = W.Batch(dims, DX, precision=W.WW_FP64)
    ar = bt.new_arena()
    fill(bt, ar, seed0=4500)
    v = bt.view(ar, 1)
    v[7, 5, 5, 5] = 0.0                       # negative pressure in patch 1
    frozen = v.clone()
    bt.step(ar)
    dts, flags = bt.dt()
    assert flags[1] > 0 and dts[1] == 0.0
    assert flags[0] == 0 and flags[2] == 0 and dts[0] > 0 and dts[2] > 0
    sl = I.interior_slices(12, 12, 12)
    assert torch.equal(bt.view(ar, 1)[sl], frozen[sl])     # left unadvanced
