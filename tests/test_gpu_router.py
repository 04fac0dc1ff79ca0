"""Learned troubled-interface router on the GPU: the MFMA MLP against the
FP64 oracle (exactly, once the oracle rounds operands to BF16 as the MFMA
inputs are; loosely without), its gradient against the oracle, Adam
training, the sampled features and weight-deviation labels against the
oracle, both forced routes of the learned sweep (all full = the plain FP32
sweep bitwise; all linear = the oracle's linear-flux right-hand side) and a
router trained on a shocked state."""
import math

import numpy as np
import pytest

from gpu_helpers import say, scaled_rhs_error
from oracle import mlp as M
from oracle import oracle as O
from paper_1808_10633_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1808_10633_amd import router as R  # noqa: E402
from paper_1808_10633_amd import wombat as W  # noqa: E402


def bf16(x):
    """Round to BF16 (nearest even), as the kernels round MFMA operands."""
    a = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    a = (a + 0x7FFF + ((a >> 16) & 1)) & 0xFFFF0000
    return a.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(theta, X):
    W1, b1, W2, b2, w3, b3 = M.unpack(theta)
    z1 = bf16(X) @ bf16(W1).T + b1
    h1 = bf16(np.maximum(z1, 0.0))
    z2 = h1 @ bf16(W2).T + b2
    return np.maximum(z2, 0.0) @ w3 + b3


def test_mlp_forward_matches_oracle():
    rng = np.random.default_rng(0)
    theta = M.init_params(1)
    theta[M.NH * M.NIN:M.NH * M.NIN + M.NH] = rng.normal(size=M.NH) * 0.1      # nonzero b1
    X = rng.uniform(-1, 1, size=(1000, 48))
    th = torch.tensor(theta, dtype=torch.float32, device="cuda")
    Xg = torch.tensor(X, dtype=torch.float32, device="cuda")
    z = W.mlp_forward(th, Xg).double().cpu().numpy()
    ze = forward_bf16(theta.astype(np.float32).astype(np.float64), X.astype(np.float32))
    zo = M.forward(theta, X)["logit"]
    e1 = np.abs(z - ze).max() / (1 + np.abs(ze).max())
    e2 = np.abs(z - zo).max() / (1 + np.abs(zo).max())
    say(f"[mlp forward] vs bf16-rounded oracle {e1:.2e}, vs fp64 oracle {e2:.2e}")
    assert e1 < 1e-5
    assert e2 < 3e-2


def grad_bf16(theta, X, t):
    """The oracle's gradient (mlp.grad's chain rule, FP64 arithmetic) with the
    operands the kernels feed to MFMA rounded to BF16: X, W1, W2, the hidden
    activations H1, the output deltas D2 and the masked hidden deltas D1.
    Returns the gradient, the loss and, per parameter, the sum of the
    absolute values of its per-sample terms (the scale of its rounding)."""
    W1, b1, W2, b2, w3, b3 = M.unpack(theta)
    Xb, W1b, W2b = bf16(X), bf16(W1), bf16(W2)
    z1 = Xb @ W1b.T + b1
    h1 = bf16(np.maximum(z1, 0.0))
    z2 = h1 @ W2b.T + b2
    h2 = np.maximum(z2, 0.0)
    z = h2 @ w3 + b3
    n = X.shape[0]
    g = (M.sigmoid(z) - t) / n
    d2 = bf16(np.outer(g, w3) * (z2 > 0))
    d1 = bf16((d2 @ W2b) * (z1 > 0))
    grad = M.pack(d1.T @ Xb, d1.sum(0), d2.T @ h1, d2.sum(0), h2.T @ g, g.sum())
    absd = M.pack(np.abs(d1).T @ np.abs(Xb), np.abs(d1).sum(0), np.abs(d2).T @ h1, np.abs(d2).sum(0),
                  h2.T @ np.abs(g), np.abs(g).sum())
    loss = float(np.mean(np.logaddexp(0.0, z) - t * z))
    return grad, loss, absd, (z1, z2)


def test_mlp_grad_matches_oracle_elementwise():
    # Samples are drawn so that no pre-activation lies within 1e-3 of zero in
    # the oracle: the kernel forms them in FP32 from the same BF16 operands
    # (error ~1e-6 of their scale), so every ReLU mask agrees.
    rng = np.random.default_rng(1)
    theta = M.init_params(2)
    theta[M.NH * M.NIN:M.NH * M.NIN + M.NH] = rng.normal(size=M.NH) * 0.1      # nonzero b1
    theta[-1] = 0.3
    theta = theta.astype(np.float32).astype(np.float64)
    X = bf16(rng.uniform(-1, 1, size=(1200, 48)).astype(np.float32))
    _, _, _, (z1, z2) = grad_bf16(theta, X, np.zeros(len(X)))
    keep = (np.abs(z1).min(1) > 1e-3) & (np.abs(z2).min(1) > 1e-3)
    X = X[keep][:777]                        # 777: six full blocks of 128 and a ragged one
    assert len(X) == 777
    t = (rng.uniform(size=777) < 0.3).astype(np.float64)
    th = torch.tensor(theta, dtype=torch.float32, device="cuda")
    g, loss = W.mlp_grad(th, torch.tensor(X, dtype=torch.float32, device="cuda"),
                         torch.tensor(t, dtype=torch.float32, device="cuda"))
    g = g.double().cpu().numpy()
    ge, le, absd, _ = grad_bf16(theta, X, t)
    go = M.grad(theta, X, t)
    # Both sides use the same BF16 operands; they differ by FP32 accumulation
    # (<= 777 * 2^-24 of the term sum) and by an operand that FP32 and FP64
    # round to neighbouring BF16 values (one BF16 step, <= 2^-7 of its term,
    # compounding once from D2 into D1).  Bound per parameter: 2^-6 of the
    # sum of its absolute terms, plus a floor.
    err = np.abs(g - ge)
    bound = 2.0 ** -6 * absd + 1e-9
    names = ("W1", "b1", "W2", "b2", "w3", "b3")
    sizes = (M.NH * M.NIN, M.NH, M.NH * M.NH, M.NH, M.NH, 1)
    o = 0
    for nm, sz in zip(names, sizes):
        sl = slice(o, o + sz)
        rel = err[sl].max() / np.abs(ge[sl]).max()
        say(f"[mlp grad] {nm}: max |gpu - bf16 oracle| {err[sl].max():.2e} ({rel:.2e} of the block max), "
            f"worst ratio to the bound {(err[sl] / bound[sl]).max():.3f}; "
            f"vs the FP64 oracle {np.abs(g[sl] - go[sl]).max() / np.abs(go[sl]).max():.2e}")
        assert (err[sl] <= bound[sl]).all(), nm
        assert rel < 1e-3, nm
        o += sz
    assert abs(float(loss) - le) < 1e-5
    assert abs(float(loss) - M.loss(theta, X, t)) < 1e-2


def test_training_learns_a_rule():
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, size=(20000, 48))
    t = ((X[:, 3] * X[:, 7] + 0.5 * X[:, 20]) > 0.1).astype(np.float64)
    Xg = torch.tensor(X, dtype=torch.float32, device="cuda")
    tg = torch.tensor(t, dtype=torch.float32, device="cuda")
    theta, hist = R.train(Xg, tg, steps=600, batch=2048, lr=3e-3, seed=0, log_every=100)
    st = R.evaluate(theta, Xg, tg)
    say(f"[train] loss {hist[0][1]:.3f} -> {hist[-1][1]:.3f}, accuracy {st['accuracy']:.3f}")
    assert hist[-1][1] < 0.5 * hist[0][1]
    assert st["accuracy"] > 0.9


def test_router_sample_matches_oracle():
    n = 12
    g = O.Grid(n, n, n, 1 / n, 1 / n, 1 / n)
    u = I.turbulence((n, n, n), mach=2.0, beta=1.0, seed=61, kmax=5).numpy().copy()
    ctx = W.Context(n, n, n, precision=W.WW_FP64)
    ug = torch.from_numpy(u).cuda()
    where = R.random_interfaces((n, n, n), 300, seed=3)
    X, dev, exs = ctx.router_sample(ug, where)
    X = X.double().cpu().numpy()
    dev = dev.double().cpu().numpy()
    exs = exs.double().cpu().numpy()
    uf = u.copy()
    O.fill_ghosts(g, uf)
    wh = where.cpu().numpy()
    ex = ed = ee = 0.0
    worst = None
    for s, (d, i, j, k) in enumerate(wh):
        t1, t2 = (d + 1) % 3, (d + 2) % 3
        perm = [0, 1 + d, 1 + t1, 1 + t2, 4 + d, 4 + t1, 4 + t2, 7]
        st = []
        for c in range(6):
            p = [i, j, k]
            p[d] = p[d] - 3 + c
            st.append(uf[perm, p[2] + 3, p[1] + 3, p[0] + 3])
        st = np.array(st)
        e = np.abs(X[s] - M.features(st)).max()
        if e > ex:
            ex, worst = e, (s, int(np.argmax(np.abs(X[s] - M.features(st)))))
        _, dv = O.interface_flux_ex(st)
        ed = max(ed, abs(dev[s] - dv))
        xo = O.flux_excess(st)
        ee = max(ee, abs(exs[s] - xo) / (1e-6 * xo + 1e-12))
    say(f"[router sample] features {ex:.2e} (sample, feature {worst}), deviation {ed:.2e}, "
        f"excess {ee:.2f} of its tolerance")
    assert ex < 1e-6 and ed < 1e-6 and ee < 1.0
    # positions outside the box read as NaN, the rest are unaffected
    bad = torch.tensor([[0, n + 1, 0, 0], [1, 0, n + 1, 0], [3, 0, 0, 0], [2, -1, 0, 0], list(wh[0])],
                       dtype=torch.int32, device="cuda")
    Xb, db, eb = ctx.router_sample(ug, bad)
    assert torch.isnan(Xb[:4]).all() and torch.isnan(db[:4]).all() and torch.isnan(eb[:4]).all()
    assert np.array_equal(Xb[4].double().cpu().numpy(), X[0]) and float(eb[4]) == float(exs[0])


def _fp32_ctx_rhs(n, u, theta=None, mode=0, thr=0.5):
    ctx = W.Context(n, n, n, precision=W.WW_FP32_MIXED, learned=1)
    if theta is not None:
        ctx.set_router(theta, thr, mode)
    ug = torch.from_numpy(u).cuda().float()
    dg = torch.zeros_like(ug)
    ctx.rhs(ug, dg)
    torch.cuda.synchronize()
    return ctx, dg


def test_learned_sweep_forced_routes():
    n = 20
    u = I.turbulence((n, n, n), mach=1.5, beta=10.0, seed=62, kmax=6).numpy().copy()
    theta = R.init_params(5)
    _, plain = _fp32_ctx_rhs(n, u)
    ctx, full = _fp32_ctx_rhs(n, u, theta, mode=1)
    assert torch.equal(plain, full)                        # same face arithmetic
    assert ctx.router_stats()[0] == 0
    ctx, lin = _fp32_ctx_rhs(n, u, theta, mode=-1)
    sm, tot, _ = ctx.router_stats()
    assert sm == tot > 0
    g = O.Grid(n, n, n, 1 / n, 1 / n, 1 / n)
    ref = O.rhs_linear(g, u)
    err, _ = scaled_rhs_error(g.interior(lin.double().cpu().numpy()), g.interior(ref), g.interior(u), 1 / n)
    say(f"[learned sweep] all-linear vs oracle linear rhs {err:.2e}")
    assert err < 2e-6


def test_routed_sweep_matches_its_two_routes():
    # the routed sweep (mode 0) with a network that calls everything troubled
    # (all interfaces through the queue and the full-WENO pass) must equal
    # the plain FP32 sweep bitwise; calling everything smooth must equal the
    # all-linear mode bitwise; a mixed routing must equal one of the two at
    # every cell whose neighbourhood is routed one way
    n = 24
    u = I.turbulence((n, n, n), mach=2.0, beta=5.0, seed=63, kmax=6).numpy().copy()
    theta = R.init_params(7)
    _, plain = _fp32_ctx_rhs(n, u)
    _, lin = _fp32_ctx_rhs(n, u, theta, mode=-1)
    hi = theta.clone()
    hi[-1] = 1e4
    ctx, r1 = _fp32_ctx_rhs(n, u, hi, mode=0)
    assert ctx.router_stats()[0] == 0
    # the queued pass and the plain sweep are separately compiled kernels of
    # the same FP32 face arithmetic: equal up to FMA contraction choices
    g = O.Grid(n, n, n, 1 / n, 1 / n, 1 / n)
    e1, _ = scaled_rhs_error(g.interior(r1.double().cpu().numpy()), g.interior(plain.double().cpu().numpy()),
                             g.interior(u), 1 / n)
    say(f"[routed sweep] all troubled (queued full WENO) vs plain FP32 sweep: {e1:.2e}")
    assert e1 < 1e-6
    lo = theta.clone()
    lo[-1] = -1e4
    ctx, r0 = _fp32_ctx_rhs(n, u, lo, mode=0)
    sm, tot, _ = ctx.router_stats()
    assert sm == tot and torch.equal(r0, lin)
    # mixed: half of the box uniform (every feature of its interfaces equal,
    # hence one logit z0, routed one way), the threshold at the median logit
    # of the other interfaces, so the turbulent half is mixed
    ctx = W.Context(n, n, n, precision=W.WW_FP32_MIXED, learned=1)
    u2 = u.copy()
    u2[:, 3:n + 3, 3:n + 3, 3:3 + n // 2] = u[:, 3:n + 3, 3:n + 3, 3:3 + n // 2].mean(axis=(1, 2, 3))[:, None, None, None]
    ug = torch.from_numpy(u2).cuda().float()
    _, plain = _fp32_ctx_rhs(n, u2)
    _, lin = _fp32_ctx_rhs(n, u2, theta, mode=-1)
    faces = []
    for d in range(3):
        lim = [n + (d == a) for a in range(3)]
        g = torch.stack(torch.meshgrid(*[torch.arange(m) for m in lim], indexing="ij"), -1).reshape(-1, 3)
        faces.append(torch.cat([torch.full((len(g), 1), d), g], 1))
    where = torch.cat(faces).to(torch.int32).cuda().contiguous()
    X, _, _ = ctx.router_sample(ug, where)
    z = W.mlp_forward(theta, X).cpu()
    wh = where.cpu().long()
    inner = (wh[:, 1] >= 3) & (wh[:, 1] <= n // 2 - 3)              # stencils inside the uniform half
    z0 = float(z[inner].max())
    assert float(z[inner].min()) == z0
    tl = float(z[~inner].median())             # splits the turbulent half
    if abs(tl - z0) < 0.01:
        tl = z0 + 0.02
    ctx.set_router(theta, 1.0 / (1.0 + math.exp(-tl)), 0)
    mix = torch.zeros_like(ug)
    ctx.rhs(ug, mix)
    torch.cuda.synchronize()
    sm, tot, _ = ctx.router_stats()
    say(f"[routed sweep] mixed routing: {sm}/{tot} smooth")
    assert 0 < sm < tot
    # per cell (periodic box): may any face touching it, or one of its 26
    # neighbours (CT reaches that far), go the other way?  Faces within 1e-4
    # of the threshold count as both.
    anyt = torch.zeros((n,) * 3, dtype=torch.bool)
    anys = torch.zeros((n,) * 3, dtype=torch.bool)
    for flag, grid in ((z > tl - 1e-4, anyt), (z < tl + 1e-4, anys)):
        sel = wh[flag]
        c = sel[:, 1:] % n                                  # face i sits between cells i-1 and i
        grid[c[:, 0], c[:, 1], c[:, 2]] = True
        c2 = sel[:, 1:].clone()
        c2[torch.arange(len(c2)), sel[:, 0]] -= 1
        c2 %= n
        grid[c2[:, 0], c2[:, 1], c2[:, 2]] = True
    def pool(g):
        gp = torch.nn.functional.pad(g[None, None].float(), (1, 1, 1, 1, 1, 1), mode="circular")
        return torch.nn.functional.max_pool3d(gp, 3, 1, 0)[0, 0] > 0
    full_only = ~pool(anys)
    lin_only = ~pool(anyt)
    sl = I.interior_slices(n, n, n)
    m, p_, l_ = mix[sl].cpu(), plain[sl].cpu(), lin[sl].cpu()
    fo = full_only.permute(2, 1, 0)                      # (x, y, z) -> (z, y, x)
    lo_ = lin_only.permute(2, 1, 0)
    say(f"  cells routed all-full {int(fo.sum())}, all-linear {int(lo_.sum())}")
    assert int(lo_.sum()) + int(fo.sum()) > 0
    assert torch.equal(m[:, lo_], l_[:, lo_])
    scale = p_.abs().amax(dim=(1, 2, 3), keepdim=True)[:, :, 0, 0]
    d = ((m[:, fo] - p_[:, fo]).abs() / scale).max() if int(fo.sum()) else torch.tensor(0.0)
    say(f"  full-only cells vs plain: {float(d):.2e} of each variable's largest |rhs|")
    assert float(d) < 1e-5


def test_routed_step_reuses_first_stage_decisions():
    # a step evaluates the network at its first stage and reuses those
    # decisions for the other three: with a network that calls everything
    # troubled (smooth) the step equals the plain (all-linear) step
    n = 20
    u = I.turbulence((n, n, n), mach=1.0, beta=10.0, seed=64, kmax=5).float().cuda().contiguous()
    theta = R.init_params(9)
    ref = W.Context(n, n, n, precision=W.WW_FP32_MIXED)
    dt = ref.cfl_dt(u)
    up = u.clone()
    ref.step(up, dt)
    hi = theta.clone()
    hi[-1] = 1e4
    ctx = W.Context(n, n, n, precision=W.WW_FP32_MIXED, learned=1)
    ctx.set_router(hi, 0.5, 0)
    ut = u.clone()
    ctx.step(ut, dt)
    g = O.Grid(n, n, n, 1 / n, 1 / n, 1 / n)
    S = np.abs(g.interior(up.double().cpu().numpy())).reshape(8, -1).max(1)
    e = float((np.abs(g.interior((ut - up).double().cpu().numpy())).reshape(8, -1).max(1) / np.maximum(S, 1e-30)).max())
    say(f"[routed step] all troubled vs plain step: {e:.2e}")
    assert e < 1e-6 and ctx.router_stats()[2] == 0
    lo = theta.clone()
    lo[-1] = -1e4
    ctx.set_router(lo, 0.5, -1)
    ul = u.clone()
    ctx.step(ul, dt)
    ctx.set_router(lo, 0.5, 0)
    ur = u.clone()
    ctx.step(ur, dt)
    torch.cuda.synchronize()
    assert ctx.router_stats()[2] == 0 and torch.equal(ur, ul)


def blast_tube(n):
    """1-D periodic tube, pressure 100 on the left half and 0.01 on the right,
    rho = 1, at rest, no field: the linear flux drives the pressure negative
    within the first RK4 step, full characteristic WENO does not."""
    x = torch.arange(n, dtype=torch.float64)
    p = torch.where(x < n // 2, 100.0, 0.01).reshape(1, 1, n)
    z = torch.zeros_like(p)
    u = torch.zeros(I.padded_shape(n, 1, 1), dtype=torch.float64)
    u[I.interior_slices(n, 1, 1)] = I.conserved(torch.ones_like(p), [z, z, z], [z, z, z], p, 5.0 / 3.0)
    return u.float().cuda()


def test_routed_step_falls_back_to_full_weno():
    n = 64
    theta = R.init_params(3)
    theta[-1] = -1e4                                   # the network calls every interface smooth
    ref = blast_tube(n)
    plain = W.Context(n, precision=W.WW_FP32_MIXED)
    dt = plain.cfl_dt(ref)
    plain.step(ref, dt)
    ctx = W.Context(n, precision=W.WW_FP32_MIXED, learned=1)
    ctx.set_router(theta, 0.5, 0)
    u = blast_tube(n)
    ctx.step(u, dt)
    torch.cuda.synchronize()
    sm, tot, fb = ctx.router_stats()
    say(f"[fallback] fallbacks {fb}, smooth in the last stage {sm}/{tot}")
    assert fb == 1 and sm == 0                         # redone with full WENO everywhere
    assert torch.equal(u, ref)
    # without the fallback (all-linear mode) the same step is non-physical
    ctx.set_router(theta, 0.5, -1)
    u = blast_tube(n)
    ctx.step(u, dt)
    with pytest.raises(W.WenoError):
        ctx.cfl_dt(u)


def shocked_state(n, seed, steps, kmax=8.0):
    """Supersonic turbulence (rms Mach 3, beta 10, 10 % compressive energy,
    log-normal density sigma 0.5) advanced `steps` FP32 full-WENO steps."""
    u = I.turbulence((n, n, n), mach=3.0, beta=10.0, seed=seed, compressive_fraction=0.1,
                     lognormal_sigma=0.5, kmax=kmax, device="cuda").float().contiguous()
    ctx = W.Context(n, n, n, precision=W.WW_FP32_MIXED, learned=1)
    for _ in range(steps):
        ctx.step(u, 0.0)
    torch.cuda.synchronize()
    return ctx, u


def test_router_trained_on_shocked_state():
    n = 256
    say("[router] training on a shocked 256^3 state")
    ctx, u = shocked_state(n, 5001, 100)
    X, dev, ex, t = R.sample(ctx, u, 120000, seed=7)
    frac = float(t.mean())
    say(f"  troubled fraction {frac:.3f}")
    assert 0.01 < frac < 0.99
    theta, hist = R.train(X[:100000], t[:100000], steps=1500, batch=4096, lr=2e-3, seed=1, log_every=500)
    st = R.evaluate(theta, X[100000:], t[100000:])
    thr = R.choose_threshold(theta, X[:100000], t[:100000], max_false_smooth=0.02)
    st2 = R.evaluate(theta, X[100000:], t[100000:], thr)
    say(f"  loss {hist[0][1]:.3f} -> {hist[-1][1]:.3f}; held-out accuracy {st['accuracy']:.3f}; "
        f"threshold {thr:.3g}: false-smooth {st2['false_smooth_rate']:.3f}, "
        f"predicted troubled {st2['predicted_troubled_fraction']:.3f}")
    ent = -(frac * math.log(frac) + (1 - frac) * math.log(1 - frac))     # loss of a constant guess
    assert hist[-1][1] < 0.8 * ent
    assert st["accuracy"] > max(frac, 1 - frac)
    assert st2["false_smooth_rate"] < 0.06
    # learned right-hand side: closer to full WENO than the all-linear one
    full = torch.zeros_like(u)
    ctx.rhs(u, full)
    ctx.set_router(theta, thr, 0)
    lrn = torch.zeros_like(u)
    ctx.rhs(u, lrn)
    sm, tot, _ = ctx.router_stats()
    ctx.set_router(theta, thr, -1)
    lin = torch.zeros_like(u)
    ctx.rhs(u, lin)
    torch.cuda.synchronize()
    sl = I.interior_slices(n, n, n)
    e_l = float((lrn[sl] - full[sl]).abs().mean() / full[sl].abs().mean())
    e_0 = float((lin[sl] - full[sl]).abs().mean() / full[sl].abs().mean())
    say(f"  smooth fraction {sm / tot:.3f}; rhs L1 vs full: learned {e_l:.2e}, all-linear {e_0:.2e}")
    assert sm > 0 and e_l < e_0
