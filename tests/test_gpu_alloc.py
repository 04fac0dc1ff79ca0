"""No device or pinned-host allocation after init: every call of a context
and of a batch after its init -- routing set-up, routed and plain steps,
stages, right-hand sides, reductions, kernel timing, the batched autotuner,
eager and graph-replayed batched steps -- leaves the library's allocation
count unchanged (the condition for capturing stages in HIP graphs)."""
import numpy as np
import pytest

from gpu_helpers import say
from paper_1808_10633_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import mlp as M  # noqa: E402
from paper_1808_10633_amd import router as R  # noqa: E402
from paper_1808_10633_amd import wombat as W  # noqa: E402


def test_no_allocation_after_init(tmp_path):
    torch.cuda.set_device(0)
    n = 24
    u = I.turbulence((n, n, n), mach=1.0, beta=10.0, seed=91, kmax=6).float().cuda().contiguous()
    ctx = W.Context(n, n, n, precision=W.WW_FP32_MIXED, learned=1)
    dims = [(16, 24, 16), (24, 16, 32), (16, 16, 16)]
    bt = W.Batch(dims, 1.0 / 32)
    ar = bt.new_arena()
    for p, d in enumerate(dims):
        bt.view(ar, p).copy_(I.turbulence(d, mach=1.0, beta=10.0, seed=92 + p, dx=1.0 / 32, kmax=4).float())
    theta = torch.tensor(M.init_params(3), dtype=torch.float32, device="cuda")
    where = R.random_interfaces((n, n, n), 64, seed=1)
    u0 = u.clone()
    acc = torch.zeros_like(u)
    out = torch.zeros_like(u)
    torch.cuda.synchronize()
    before = W.alloc_count()
    ctx.set_router(theta, 0.5, 0)
    ctx.step(u, 0.0)
    ctx.router_stats()
    ctx.set_router(theta, 0.5, -1)
    ctx.step(u, 0.0)
    ctx.set_router(None)
    dt = ctx.cfl_dt(u)
    ctx.step(u, dt)
    u1 = u.clone()
    ctx.stage(0, dt, u1, u1, acc, out)
    ctx.rhs(u, out)
    ctx.sums(u)
    ctx.divb(u)
    ctx.time_kernels(u, reps=2)
    ctx.router_sample(u, where)
    bt.autotune(ar, str(tmp_path / "tune.jsonl"))
    bt.step(ar)
    bt.graph_steps(ar, 2)
    bt.dt()
    torch.cuda.synchronize()
    after = W.alloc_count()
    say(f"[alloc] library allocations: {before} after init, {after} after the calls")
    assert after == before
    assert torch.isfinite(u).all() and torch.isfinite(ar).all()
    del u0
    bt.close()
    ctx.close()


def test_set_router_needs_learned_buffers():
    ctx = W.Context(16, 16, 16, precision=W.WW_FP32_MIXED)
    theta = torch.zeros(W.mlp_param_count(), dtype=torch.float32, device="cuda")
    with pytest.raises(W.WenoError, match="learned") as e:
        ctx.set_router(theta, 0.5)
    assert e.value.code == W.WW_ERR_STATE
    ctx.set_router(None)        # switching routing off needs nothing
    ctx.close()


def test_autotuner_leaves_the_arena_unchanged_and_keeps_dt():
    dims = [(16, 16, 24), (24, 16, 16)]
    bt = W.Batch(dims, 1.0 / 32)
    ar = bt.new_arena()
    for p, d in enumerate(dims):
        bt.view(ar, p).copy_(I.turbulence(d, mach=1.0, beta=10.0, seed=95 + p, dx=1.0 / 32, kmax=4).float())
    ref = ar.clone()
    ms = bt.autotune(ar, None)
    torch.cuda.synchronize()
    assert ms > 0
    assert torch.equal(ar, ref)
    dts, flags = bt.dt()
    # the tuner recomputed each patch's dt from the arena: a step takes the same
    bt.step(ar)
    dts2, _ = bt.dt()
    assert np.array_equal(dts, dts2) and (flags == 0).all()
    bt.close()
