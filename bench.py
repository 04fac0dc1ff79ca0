"""Benchmark of the WENO5-MHD stage library on one MI355X.

Workload: decaying MHD turbulence in a periodic 512^3 box (rms Mach 1.0,
plasma beta 100, gamma 5/3, the turbulence generator of the precision-form
configuration), advanced with full FP64 RK4 steps (CFL time step, 4 stages of
ghost fill + x/y/z characteristic WENO sweeps + flux difference/CT/RK update)
through the C ABI.  Inputs are resident in HBM before the timed region.

Prints one JSON line: zone-stage updates/s over `--steps` timed steps, the
roofline of the dominant kernel (the characteristic sweep, VALU-bound, FP64
vector peak) from HIP-event kernel timings, and the serial CPU oracle timed
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "zone-stage updates/s (WENO5-MHD 512^3) FP64 vs FP32/learned at stated L1 err; %HBM"

FP64_VECTOR_PEAK_TFLOPS = 78.6      # MI355X FP64 vector peak
FP32_VECTOR_PEAK_TFLOPS = 157.3     # MI355X FP32 vector peak (packed)

# HBM bytes per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE runs (scaled
# by a 1 GiB copy; see profiles/), valid only for the kernel source they were
# taken on: sha256 of ww_sweep.hip + ww_sweep_dev.h (sweeps) or ww_update.hip
# + ww_update_dev.h (update).
MEASURED_TRAFFIC = {
    # y sweep (the VALU roofline's kernel) and the fused x sweep
    ("b97c660155bc5f2d", "fp64", 512): {"read": 9.406e9, "write": 9.05e9,
                                      "profile": "profiles/fp64_512_turbulence_trace_and_hbm.md"},
    ("b97c660155bc5f2d", "fp32", 512): {"read": 4.788e9, "write": 4.711e9,
                                      "profile": "profiles/fp32_512_turbulence_trace_and_hbm.md"},
    ("b97c660155bc5f2d", "fp64_xfused", 512): {"read": 31.23e9, "write": 11.64e9,
                                             "profile": "profiles/fp64_512_turbulence_trace_and_hbm.md"},
    ("b97c660155bc5f2d", "fp32_xfused", 512): {"read": 15.24e9, "write": 5.837e9,
                                             "profile": "profiles/fp32_512_turbulence_trace_and_hbm.md"},
}
MEASURED_UPDATE_TRAFFIC = {
    # B-only update, mean over the profiled launches (RK stage forms and L(U))
    ("cf6b38782c5af04b", "fp64", 512): {"read": 11.8e9, "write": 5.585e9,
                                      "profile": "profiles/fp64_512_turbulence_trace_and_hbm.md"},
    ("cf6b38782c5af04b", "fp32", 512): {"read": 5.73e9, "write": 2.818e9,
                                      "profile": "profiles/fp32_512_turbulence_trace_and_hbm.md"},
}

# HBM bytes per stage launch of the batched kernel on the 4096-patch set
# (autotuned faces per y/z tile -> read, write), from the same counter runs,
# valid only for the batched source they were taken on (sha256 of
# ww_batch.hip, ww_batch.h, ww_sweep_dev.h, ww_update_dev.h, ww_internal.h).
MEASURED_BATCH_TRAFFIC = {
    ("357f8b2041d60ec0", 4096, 4): (85.48e9, 32.26e9),
    ("357f8b2041d60ec0", 4096, 8): (79.57e9, 32.72e9),
    ("357f8b2041d60ec0", 4096, 12): (81.07e9, 31.47e9),
    ("357f8b2041d60ec0", 4096, 16): (79.07e9, 32.45e9),
}
BATCH_TRAFFIC_PROFILE = "profiles/batched_4096_patches_hbm.md"


def batch_source_hash():
    import hashlib
    d = os.path.join(ROOT, "paper_1808_10633_amd", "csrc")
    src = b"".join(open(os.path.join(d, f), "rb").read()
                   for f in ("ww_batch.hip", "ww_batch.h", "ww_sweep_dev.h", "ww_update_dev.h", "ww_internal.h"))
    return hashlib.sha256(src).hexdigest()[:16]


def _source_hash(files):
    import hashlib
    d = os.path.join(ROOT, "paper_1808_10633_amd", "csrc")
    src = b"".join(open(os.path.join(d, f), "rb").read() for f in files)
    return hashlib.sha256(src).hexdigest()[:16]


def sweep_source_hash():
    return _source_hash(("ww_sweep.hip", "ww_sweep_dev.h"))


def update_source_hash():
    return _source_hash(("ww_update.hip", "ww_update_dev.h"))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 precision form")
    ap.add_argument("--batch-patches", type=int, default=4096,
                    help="patches of the batched form (0 skips it)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-router form")
    ap.add_argument("--fp32-box", type=int, default=0,
                    help="only the FP32 form on an N^3 box of the default turbulence (its own JSON line): "
                         "sizes whose FP64 run does not fit one GPU")
    ap.add_argument("--precision-box", type=int, default=0,
                    help="only the precision form against an FP64 run on an N^3 box (own JSON line), both "
                         "in z-slab mode: 1024^3 FP64 fits one GPU that way")
    ap.add_argument("--slab-planes", type=int, default=64, help="slab thickness of --precision-box")
    ap.add_argument("--patch-sweep", action="store_true",
                    help="only run the batched form at uniform patch sizes 8^3..64^3 (one JSON line)")
    ap.add_argument("--ablation", action="store_true",
                    help="scheme variants (WENO-Z weights, SSP-RK3): cost at --n and robustness on shocked "
                         "turbulence (own JSON line)")
    ap.add_argument("--abl-steps", type=int, default=300)
    ap.add_argument("--learned-n", type=int, default=512)
    ap.add_argument("--train-n", type=int, default=256)
    ap.add_argument("--pre-steps", type=int, default=200,
                    help="full-WENO FP32 steps that shock the learned-form turbulence")
    ap.add_argument("--learned-steps", type=int, default=50)
    ap.add_argument("--train-steps", type=int, default=3000)
    ap.add_argument("--cpu-n", type=int, default=112, help="box of the single-core oracle sample")
    ap.add_argument("--cpu-omp-n", type=int, default=192, help="box of the all-core oracle sample")
    ap.add_argument("--compare-steps", type=int, default=50,
                    help="steps after which the FP32 form is compared with the FP64 run")
    ap.add_argument("--config2-steps", type=int, default=100,
                    help="steps of the 256^3 subsonic FP64 turbulence form (0 skips it)")
    ap.add_argument("--reps", type=int, default=5, help="launches per kernel for the event timing")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def copy_calibration(mib):
    """A plain copy kernel of known size: reads and writes mib MiB once."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_mib": mib, "bytes_read": n * 8, "bytes_written": n * 8}), flush=True)


HBM_PEAK = 8.0e12   # MI355X HBM3E, bytes/s


KERNELS = ("ghosts", "sweep_x", "sweep_y", "sweep_z", "update_stage", "cfl", "update_rhs")


def kernel_table(ms, ms_per_step, stages=4):
    """Event-timed kernels of a step and their sum against the step time."""
    km = dict(zip(KERNELS, ms))
    per_step = km["cfl"] + stages * sum(km[k] for k in ("ghosts", "sweep_x", "sweep_y", "sweep_z", "update_stage"))
    return {"kernel_ms": km, "kernels_ms_per_step": round(per_step, 3),
            "kernels_frac_of_step": round(per_step / ms_per_step, 4)}


def roofline_sweep(ms_y, n, prec, opcount, peak):
    """VALU roofline of the y sweep (the characteristic WENO flux of every
    interface of one direction) from its event-timed launch."""
    nface = (n + 1) * (n + 2) * (n + 2)
    fpi = opcount.flops_per_interface()
    achieved = fpi * nface / (ms_y * 1e-3) / 1e12
    dense = opcount.DENSE_FLOPS_PER_INTERFACE * nface / (ms_y * 1e-3) / 1e12
    tr = MEASURED_TRAFFIC.get((sweep_source_hash(), prec, n))
    traffic = (tr["read"] + tr["write"]) if tr else None
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": traffic, "traffic_unit": "bytes/launch",
            "traffic_source": tr["profile"] if tr else None,
            "hbm_TBps": round(traffic / (ms_y * 1e-3) / 1e12, 3) if tr else None,
            "hbm_frac": round(traffic / (ms_y * 1e-3) / HBM_PEAK, 4) if tr else None,
            "kernel": ("sweep_yz_kernel<1,32,double>" if prec == "fp64" else "sweep_kernel<1,8,float>") + " (y sweep)",
            "ms": ms_y, "flop_per_interface": fpi, "interfaces_per_launch": nface,
            "frac_dense_count": round(dense / peak, 4),
            "dense_flop_per_interface": opcount.DENSE_FLOPS_PER_INTERFACE}


def roofline_update(ms_u, n, prec, opcount, fused_x=True):
    """HBM roofline of the update in its stage forms: algorithmic bytes per
    launch (averaged over the four stage forms; with the fused x sweep the
    update carries constrained transport and B only) over the event-timed
    launch."""
    es = 8 if prec == "fp64" else 4
    bpc = opcount.update_bytes_per_cell(es, fused_x=fused_x)
    nbytes = bpc * n ** 3
    achieved = nbytes / (ms_u * 1e-3) / 1e9
    tr = MEASURED_UPDATE_TRAFFIC.get((update_source_hash(), prec, n))
    traffic = (tr["read"] + tr["write"]) if tr else None
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": round(achieved * 1e9 / HBM_PEAK, 4), "traffic": traffic, "traffic_unit": "bytes/launch",
            "traffic_source": tr["profile"] if tr else None,
            "kernel": f"update_march_kernel<{'double' if es == 8 else 'float'}, {'true' if fused_x else 'false'}, "
                      f"false> (RK stage forms{', B only' if fused_x else ''})",
            "ms": ms_u, "algorithmic_bytes_per_cell": bpc, "cells_per_launch": n ** 3}


def roofline_xfused(ms_x, n, prec, opcount, peak):
    """The x sweep with the rho, m, E update fused in: it does the sweep's
    flux arithmetic and moves the hydro update's data.  HBM roofline on its
    algorithmic bytes per launch (the bound it is closer to), with the VALU
    fraction of its flux arithmetic beside it."""
    es = 8 if prec == "fp64" else 4
    bpc = opcount.fused_x_bytes_per_cell(es)
    nbytes = bpc * n ** 3
    achieved = nbytes / (ms_x * 1e-3) / 1e9
    nface = (n + 1) * (n + 2) * (n + 2)
    tflops = opcount.flops_per_interface() * nface / (ms_x * 1e-3) / 1e12
    tr = MEASURED_TRAFFIC.get((sweep_source_hash(), prec + "_xfused", n))
    traffic = (tr["read"] + tr["write"]) if tr else None
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": round(achieved * 1e9 / HBM_PEAK, 4), "traffic": traffic, "traffic_unit": "bytes/launch",
            "traffic_source": tr["profile"] if tr else None,
            "measured_hbm_frac": round(traffic / (ms_x * 1e-3) / HBM_PEAK, 4) if tr else None,
            "kernel": f"sweep_xfused_kernel<{'double' if es == 8 else 'float'}> (x sweep + rho, m, E update, "
                      "RK stage forms)",
            "ms": ms_x, "algorithmic_bytes_per_cell": bpc, "cells_per_launch": n ** 3,
            "valu_achieved_tflops": round(tflops, 3), "valu_frac": round(tflops / peak, 4)}


def rooflines(ms, n, prec, opcount, peak, fused_x=True):
    """Rooflines of the sweep (y), the fused x sweep and the update; the
    dominant kernel is the one with the largest time per step (each sweep
    direction and the update run once per stage)."""
    sweep = roofline_sweep(ms[2], n, prec, opcount, peak)
    upd = roofline_update(ms[4], n, prec, opcount, fused_x)
    xf = roofline_xfused(ms[1], n, prec, opcount, peak) if fused_x else None
    longest = max(("sweep_x", ms[1]), ("sweep_y", ms[2]), ("sweep_z", ms[3]), ("update_stage", ms[4]),
                  key=lambda t: t[1])[0]
    dom = {"update_stage": upd, "sweep_x": xf if fused_x else sweep}.get(longest, sweep)
    out = {"sweep_y": sweep, "update": upd}
    if xf:
        out["sweep_x_fused"] = xf
    return dict(dom, dominant=longest), out


def batched_form(a, wombat, inputs, opcount):
    """Batched form: independent periodic patches, edges drawn uniformly from
    {16,24,32,48,64} per axis (seed 4000), cell width 1/64, each an own
    turbulence realisation (rms Mach U[0.3,2], beta log-uniform in [1,1e4],
    seed 4000+p), FP32; one persistent launch per RK stage, whole steps
    replayed from a HIP graph, launch shape autotuned."""
    import numpy as np
    import tempfile
    import torch
    rng = np.random.default_rng(4000)
    npatch = a.batch_patches
    dims = [tuple(int(v) for v in rng.choice([16, 24, 32, 48, 64], size=3)) for _ in range(npatch)]
    machs = rng.uniform(0.3, 2.0, size=npatch)
    betas = 10 ** rng.uniform(0.0, 4.0, size=npatch)
    bt = wombat.Batch(dims, 1.0 / 64, precision=wombat.WW_FP32_MIXED)
    ar = bt.new_arena()
    t0 = time.perf_counter()
    for p, d in enumerate(dims):
        u = inputs.turbulence(d, mach=float(machs[p]), beta=float(betas[p]), seed=4000 + p,
                              dx=1.0 / 64, device="cuda")
        bt.view(ar, p).copy_(u.float())
    torch.cuda.synchronize()
    print(f"[bench] {npatch} patches generated in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    cache = os.path.join(tempfile.mkdtemp(), "batch_tune.jsonl")
    tune_ms = bt.autotune(ar, cache)
    ft, bpc, nblocks = bt.shape()
    bt.graph_steps(ar, a.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt.graph_steps(ar, a.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    dts, flags = bt.dt()
    zones = sum(x * y * z for x, y, z in dims)
    faces = sum((x + 1) * (y + 2) * (z + 2) + (x + 2) * (y + 1) * (z + 2) + (x + 2) * (y + 2) * (z + 1)
                for x, y, z in dims)
    stage_ms = el / (4 * a.steps) * 1e3
    achieved = opcount.flops_per_interface() * faces / (stage_ms * 1e-3) / 1e12
    tr = MEASURED_BATCH_TRAFFIC.get((batch_source_hash(), npatch, ft))
    traffic = sum(tr) if tr else None
    res = {"value": zones * 4 * a.steps / el, "unit": "zone-stage updates/s",
           "ms_per_step": el / a.steps * 1e3, "dtype": "f32 (f64 islands)",
           "patches": npatch, "interior_zones": zones, "nonphysical_patches": int((flags > 0).sum()),
           "dt_min": float(dts.min()), "dt_max": float(dts.max()),
           "launch": {"faces_per_tile": ft, "blocks_per_cu": bpc, "blocks": nblocks,
                      "autotune_best_step_ms": tune_ms, "graph": True},
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                        "traffic": traffic, "traffic_unit": "bytes/launch",
                        "traffic_source": BATCH_TRAFFIC_PROFILE if tr else None,
                        "hbm_TBps": round(traffic / (stage_ms * 1e-3) / 1e12, 3) if tr else None,
                        "hbm_frac": round(traffic / (stage_ms * 1e-3) / HBM_PEAK, 4) if tr else None,
                        "kernel": "batch_stage_kernel<FT,float> (whole stage)",
                        "flop_per_interface": opcount.flops_per_interface(),
                        "interfaces_per_launch": faces, "kernel_ms": stage_ms}}
    del bt, ar
    return res


def fp32_box(a, wombat, inputs, opcount):
    """The FP32 form alone on an N^3 box of the default turbulence recipe (rms
    Mach 1, beta 100, seed 1003), its own CFL dt every step: throughput,
    event-timed kernels and the drift of the FP64 sums.  At 1024^3 the FP32
    arrays (four states and three face-flux buffers, ~230 GB) fit one GPU; the
    FP64 run at that size does not, so there is no FP64 comparison here."""
    import torch
    n = a.fp32_box
    u = inputs.turbulence((n, n, n), mach=1.0, beta=100.0, seed=1003, device="cuda")
    u32 = u.float().contiguous()
    del u
    torch.cuda.empty_cache()
    print(f"[bench] {n}^3 FP32 turbulence ready", file=sys.stderr, flush=True)
    ctx = wombat.Context(n, n, n, precision=wombat.WW_FP32_MIXED, cfl=0.4)
    s0 = ctx.sums(u32)
    for _ in range(a.warmup):
        ctx.step(u32, 0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        ctx.step(u32, 0.0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s1 = ctx.sums(u32)
    ms = ctx.time_kernels(u32, reps=a.reps)
    ifaces = (n + 1) * (n + 2) ** 2
    achieved = opcount.flops_per_interface() * ifaces / (ms[2] * 1e-3) / 1e12
    res = {"n": n, "value": n ** 3 * 4 * a.steps / el, "unit": "zone-stage updates/s",
           "ms_per_step": el / a.steps * 1e3, "steps": a.steps, "warmup": a.warmup,
           "dtype": "f32 (f64 islands)",
           "kernel_ms": dict(zip(KERNELS, ms)),
           "y_sweep_tflops": round(achieved, 3), "y_sweep_frac_fp32_peak": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
           "mass_energy_rel_drift": [abs(s1[v] - s0[v]) / abs(s0[v]) for v in (0, 7)],
           "device_memory_gb": round(torch.cuda.mem_get_info()[1] / 1e9, 1)}
    del ctx, u32
    return res


def precision_box(a, wombat, inputs):
    """The precision form against FP64 on an N^3 box of the default turbulence
    recipe (rms Mach 1, beta 100, seed 1003): compare_steps FP64 steps with
    their CFL dt, then the FP32 form replaying those dt from the same initial
    state; L1 and Linf of every variable (relative to the FP64 field's mean
    and largest magnitude) after the last step.  Both run in z-slab mode
    (slab_planes): at 1024^3 the FP64 state, its stage state and accumulator
    (3 x 69.9 GB) and one slab's face fluxes fit one GPU, where the whole-box
    face fluxes would not."""
    import torch
    n = a.precision_box
    nst = a.compare_steps

    def ic():
        u = inputs.turbulence((n, n, n), mach=1.0, beta=100.0, seed=1003, device="cuda")
        torch.cuda.empty_cache()
        return u

    def run(u, precision, dts, label):
        ctx = wombat.Context(n, n, n, precision=precision, cfl=0.4, slab_planes=a.slab_planes)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(nst):
            if dts is None:
                dts_out.append(ctx.step(u, 0.0))
            else:
                ctx.cfl_dt(u)
                ctx.step(u, dts[i])
            if (i + 1) % 5 == 0:
                torch.cuda.synchronize()
                print(f"[bench] {label} step {i + 1}/{nst}, {time.perf_counter() - t0:.1f} s",
                      file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ms = ctx.time_kernels(u, reps=2)
        mem = torch.cuda.mem_get_info()
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
        return {"value": n ** 3 * 4 * nst / el, "ms_per_step": el / nst * 1e3,
                "kernel_ms_per_stage_all_slabs": dict(zip(KERNELS, ms)),
                "device_memory_in_use_gb": round((mem[1] - mem[0]) / 1e9, 1)}

    dts_out = []
    u64 = ic()
    # the FP32 run's initial state waits in host memory (regenerating it next
    # to the FP64 result would not fit: the generator's FFTs take ~150 GB)
    host32 = u64.float().cpu()
    torch.cuda.empty_cache()
    print(f"[bench] {n}^3 FP64 initial state ready", file=sys.stderr, flush=True)
    r64 = run(u64, wombat.WW_FP64, None, "fp64")
    u32 = host32.cuda()
    del host32
    r32 = run(u32, wombat.WW_FP32_MIXED, dts_out, "fp32")
    l1, linf = [], []
    g = 3
    for v in range(8):
        dsum = dmax = rsum = rmax = 0.0
        for k0 in range(0, n, 64):
            sl = (v, slice(g + k0, g + min(k0 + 64, n)), slice(g, g + n), slice(g, g + n))
            ref = u64[sl]
            d = (u32[sl].double() - ref).abs()
            dsum += float(d.sum())
            dmax = max(dmax, float(d.max()))
            rsum += float(ref.abs().sum())
            rmax = max(rmax, float(ref.abs().max()))
        if rmax > 0:
            l1.append(dsum / rsum)
            linf.append(dmax / rmax)
    return {"n": n, "steps": nst, "slab_planes": a.slab_planes, "fp64": r64, "fp32_mixed": r32,
            "speedup_fp32_vs_fp64": r32["value"] / r64["value"],
            "l1_rel_vs_fp64": l1, "linf_rel_vs_fp64": linf,
            "l1_rel_vs_fp64_max_var": max(l1), "linf_rel_vs_fp64_max_var": max(linf),
            "unit": "zone-stage updates/s",
            "workload": f"decaying MHD turbulence {n}^3 periodic, rms Mach 1.0, beta 100, seed 1003; FP32 form "
                        f"replays the FP64 run's CFL-0.4 steps"}


def patch_sweep(a, wombat, inputs):
    """Batched form at uniform patch edges 4..72, about 2^26 interior zones
    each (the GPU counterpart of a patch-size study): every patch holds the
    same periodic turbulence realisation (rms Mach 1, beta 100; modes up to
    |k|/2pi = 8, or e/2 - 1 on patches under 8 cells), FP32, autotuned
    launch shape, graph-replayed steps."""
    import tempfile
    import torch
    rows = []
    for e in (4, 6, 8, 12, 16, 24, 32, 48, 64, 72):
        npatch = max(1, (1 << 26) // e ** 3)
        bt = wombat.Batch([(e, e, e)] * npatch, 1.0 / e, precision=wombat.WW_FP32_MIXED)
        ar = bt.new_arena()
        # modes 2 <= |k|/2pi <= 8; patches under 8 cells keep |k|/2pi <= e/2 - 1
        # (the generator's default band leaves them without a random field)
        kmax = 8.0 if e >= 8 else e / 2 - 1
        u = inputs.turbulence((e, e, e), mach=1.0, beta=100.0, seed=4000, dx=1.0 / e, kmin=min(2.0, kmax),
                              kmax=kmax, device="cuda").float()
        # equal patches sit at equal strides in the arena: one strided copy
        stride = bt.offsets[1] - bt.offsets[0] if npatch > 1 else u.numel()
        assert all(bt.offsets[p] == bt.offsets[0] + p * stride for p in range(npatch))
        torch.as_strided(ar, (npatch, u.numel()), (stride, 1), bt.offsets[0]).copy_(
            u.reshape(1, -1).expand(npatch, -1))
        torch.cuda.synchronize()
        cache = os.path.join(tempfile.mkdtemp(), "sweep_tune.jsonl")
        bt.autotune(ar, cache)
        ft, bpc, nb = bt.shape()
        bt.graph_steps(ar, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bt.graph_steps(ar, a.steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        zones = npatch * e ** 3
        rows.append({"edge": e, "patches": npatch, "zones": zones, "value": zones * 4 * a.steps / el,
                     "ms_per_step": el / a.steps * 1e3, "faces_per_tile": ft, "blocks_per_cu": bpc})
        print(f"[bench] patch sweep {e}^3 x {npatch}: {rows[-1]['value']:.3e} zone-stage/s",
              file=sys.stderr, flush=True)
        del bt, ar
        torch.cuda.empty_cache()
    return rows


def shocked_turbulence(n, seed, wombat, inputs, pre, snaps=(), learned=0):
    """Supersonic turbulence (rms Mach 3, beta 10, 10 % of the kinetic energy
    compressive, log-normal density sigma 0.5, p = 1), advanced `pre` full
    characteristic WENO FP32 steps at CFL 0.4.  Yields (step, context, state)
    after each step listed in snaps and at the end; learned=1 gives the
    context the router's buffers."""
    u = inputs.turbulence((n, n, n), mach=3.0, beta=10.0, seed=seed, compressive_fraction=0.1,
                          lognormal_sigma=0.5, device="cuda").float().contiguous()
    ctx = wombat.Context(n, n, n, precision=wombat.WW_FP32_MIXED, cfl=0.4, learned=learned)
    for s in range(1, pre + 1):
        ctx.step(u, 0.0)
        if s in snaps and s != pre:
            yield s, ctx, u
    yield pre, ctx, u


def rel_errors(a, b, sl):
    """Per-variable relative L1 and Linf of a against b on the interior."""
    l1, linf = [], []
    for v in range(8):
        d = (a[sl][v].double() - b[sl][v].double()).abs()
        ref = b[sl][v].double().abs()
        if float(ref.max()) > 0:
            l1.append(float(d.mean() / ref.mean()))
            linf.append(float(d.max() / ref.max()))
    return max(l1), max(linf)


def learned_form(a, wombat, inputs, router):
    """Learned-router form on shocked Mach-3 turbulence.  Training: the same
    recipe at train_n^3, seeds 5001-5004, snapshots after half and all of
    the pre-steps scaled to the same physical time (pre * train_n / n steps),
    interfaces sampled at random (features and flux-excess labels from the
    library), MLP trained by the library's BF16 MFMA kernels, threshold set
    for <= 10 % false-smooth on the training set (the interfaces it routes
    smooth stay at flux excess ~1e-3: reported).  Evaluation: seed 5000 at
    learned_n^3 after pre steps; from that snapshot `learned_steps` steps of
    full WENO and of the learned route (the full run's step sizes replayed),
    compared to each other, and the all-linear route (no network) as the
    accuracy floor."""
    import torch
    t0 = time.perf_counter()
    Xs, ts = [], []
    pre_tr = max(2, round(a.pre_steps * a.train_n / a.learned_n))
    for seed in (5001, 5002, 5003, 5004):
        for step, ctx, u in shocked_turbulence(a.train_n, seed, wombat, inputs, pre_tr,
                                               snaps=(pre_tr // 2,)):
            X, _, _, t = router.sample(ctx, u, 250000, seed=seed * 10 + step)
            Xs.append(X)
            ts.append(t)
        del ctx, u
    X = torch.cat(Xs)
    t = torch.cat(ts)
    del Xs, ts
    nval = X.shape[0] // 10
    perm = torch.randperm(X.shape[0], generator=torch.Generator().manual_seed(0)).cuda()
    X, t = X[perm], t[perm]
    Xtr, ttr, Xva, tva = X[nval:], t[nval:], X[:nval], t[:nval]
    print(f"[bench] learned: {X.shape[0]} training interfaces in {time.perf_counter() - t0:.1f} s, "
          f"troubled fraction {float(t.mean()):.3f}", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    theta, hist = router.train(Xtr, ttr, steps=a.train_steps, batch=4096, lr=2e-3, seed=1,
                               log_every=max(a.train_steps // 10, 1))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    thr = router.choose_threshold(theta, Xtr, ttr, max_false_smooth=0.10)
    val = router.evaluate(theta, Xva, tva, thr)
    print(f"[bench] learned: trained in {train_s:.1f} s, loss {hist[0][1]:.3f} -> {hist[-1][1]:.3f}, "
          f"threshold {thr:.3g}", file=sys.stderr, flush=True)
    del X, t, Xtr, ttr, Xva, tva

    n = a.learned_n
    for _, ctx, u in shocked_turbulence(n, 5000, wombat, inputs, a.pre_steps, learned=1):
        pass
    Xe, deve, exe, te = router.sample(ctx, u, 250000, seed=50000)
    ev = router.evaluate(theta, Xe, te, thr, excess=exe)
    ev["weight_deviation_above_1e-2"] = float((deve > 1e-2).float().mean())
    del Xe, te, deve, exe
    snap = u.clone()
    sl = inputs.interior_slices(n, n, n)
    nsteps = a.learned_steps
    dts = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nsteps):
        dts.append(ctx.step(u, 0.0))
    torch.cuda.synchronize()
    el_full = time.perf_counter() - t0
    runs = {}
    for name, mode in (("learned", 0), ("all_linear", -1)):
        ul = snap.clone()
        ctx.set_router(theta, thr, mode)
        fb0 = ctx.router_stats()[2]
        fracs = []
        failed = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(nsteps):
            try:
                ctx.cfl_dt(ul)
                ctx.step(ul, dts[i])
            except wombat.WenoError as e:
                failed = f"step {i + 1}: {e}"
                break
            sm, tot, _ = ctx.router_stats()       # smooth share of the step's last stage
            fracs.append(sm / tot)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        if failed:
            runs[name] = {"failed": failed}
            print(f"[bench] learned: route {name} failed at {failed}", file=sys.stderr, flush=True)
            del ul
            continue
        fb = ctx.router_stats()[2] - fb0
        l1, linf = rel_errors(ul, u, sl)
        runs[name] = {"value": n ** 3 * 4 * nsteps / el, "ms_per_step": el / nsteps * 1e3,
                      "speedup_vs_full_fp32": el_full / el, "l1_rel_vs_full_max_var": l1,
                      "linf_rel_vs_full_max_var": linf, "smooth_fraction_mean": sum(fracs) / len(fracs),
                      "full_weno_fallback_steps": fb}
        print(f"[bench] learned: route {name}: {el / nsteps * 1e3:.1f} ms/step (full {el_full / nsteps * 1e3:.1f}), "
              f"L1 {l1:.2e}, smooth {sum(fracs) / len(fracs):.3f}, fallbacks {fb}", file=sys.stderr, flush=True)
        del ul
    ctx.set_router(None, 0.5, 0)
    res = {"value": runs["learned"].get("value"), "unit": "zone-stage updates/s", "dtype": "f32 + bf16 MLP",
           "workload": f"shocked turbulence {n}^3, rms Mach 3, beta 10, 10 % compressive, log-normal "
                       f"rho sigma 0.5; {a.pre_steps} full-WENO FP32 steps, then {nsteps} steps per route",
           "full_fp32": {"value": n ** 3 * 4 * nsteps / el_full, "ms_per_step": el_full / nsteps * 1e3},
           "learned": runs["learned"], "all_linear_no_network": runs["all_linear"],
           "router": {"threshold": thr, "label": f"flux excess > {router.LABEL_THRESHOLD:g}",
                      "train_interfaces": int(9 * nval), "train_pre_steps": pre_tr,
                      "train_steps": a.train_steps, "train_seconds": train_s,
                      "loss_first_last": [hist[0][1], hist[-1][1]],
                      "heldout_train_recipe": val, "eval_snapshot": ev}}
    del ctx, u, snap
    return res


ABLATIONS = (("rk4_js", "WEIGHTS_JS", "RK4", "LF_LOCAL"), ("rk4_z", "WEIGHTS_Z", "RK4", "LF_LOCAL"),
             ("ssprk3_js", "WEIGHTS_JS", "SSPRK3", "LF_LOCAL"), ("rk4_js_global_lf", "WEIGHTS_JS", "RK4", "LF_GLOBAL"))


def ablation(a, wombat, inputs):
    """Scheme variants on the single-grid operator: the paper's choice
    (weights of eq. (3), classical RK4, per-stencil LF speeds), WENO-Z weights
    (Borges et al. 2008, exponent 1), SSP-RK3 (Shu & Osher 1988) and global
    LF speeds per sweep.  Cost: timed steps and
    event-timed kernels at n^3 on the rms-Mach-1 turbulence of the default
    line, both precisions.  Robustness (FP64): the shocked turbulence recipe
    (beta 10, 10 % compressive, log-normal density sigma 0.5, seed 6000) at
    rms Mach 3, 6 and 10 on 64^3..256^3, each run up to `abl_steps` CFL-0.4
    steps (every variant takes the same CFL time step rule); a run fails at the
    step whose CFL reduction finds rho <= 0, p <= 0 or a non-finite value."""
    import torch
    n = a.n
    cost = {}
    for prec, dt_ in (("fp64", torch.float64), ("fp32", torch.float32)):
        P = wombat.WW_FP64 if prec == "fp64" else wombat.WW_FP32_MIXED
        for name, wk, ik, lk in ABLATIONS:
            u = inputs.turbulence((n, n, n), mach=1.0, beta=100.0, seed=1003, device="cuda").to(dt_).contiguous()
            ctx = wombat.Context(n, n, n, precision=P, cfl=0.4, weights=getattr(wombat, wk),
                                 integrator=getattr(wombat, ik), lf_speed=getattr(wombat, lk))
            for _ in range(a.warmup):
                ctx.step(u, 0.0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(a.steps):
                ctx.step(u, 0.0)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            ms = ctx.time_kernels(u, reps=a.reps)
            stages = 3 if ik == "SSPRK3" else 4
            cost[f"{prec}_{name}"] = {"zone_steps_per_s": n ** 3 * a.steps / el,
                                      "zone_stage_updates_per_s": n ** 3 * stages * a.steps / el,
                                      "ms_per_step": el / a.steps * 1e3, "sweep_ms_xyz": ms[1:4],
                                      "update_ms": ms[4]}
            print(f"[bench] ablation cost {prec} {name}: {el / a.steps * 1e3:.1f} ms/step, "
                  f"sweeps {sum(ms[1:4]):.2f} ms", file=sys.stderr, flush=True)
            del ctx, u
            torch.cuda.empty_cache()
    runs = []
    for m in (3.0, 6.0, 10.0):
        for e in (64, 128, 256):
            row = {"precision": "fp64", "mach": m, "n": e}
            for name, wk, ik, lk in ABLATIONS:
                u = inputs.turbulence((e, e, e), mach=m, beta=10.0, seed=6000, compressive_fraction=0.1,
                                      lognormal_sigma=0.5, device="cuda").contiguous()
                ctx = wombat.Context(e, e, e, precision=wombat.WW_FP64, cfl=0.4, weights=getattr(wombat, wk),
                                     integrator=getattr(wombat, ik), lf_speed=getattr(wombat, lk))
                t, s, fail = 0.0, 0, None
                while s < a.abl_steps:
                    s += 1
                    try:
                        t += ctx.step(u, 0.0)
                    except wombat.WenoError as err:
                        if err.code != -5:
                            raise
                        fail = s
                        break
                row[name] = {"failed_at_step": fail, "t_reached": t, "steps": s}
                del ctx, u
            print(f"[bench] ablation Mach {m:g} {e}^3: " +
                  ", ".join(f"{k} {row[k]['failed_at_step']} (t {row[k]['t_reached']:.5f})" for k, *_ in ABLATIONS),
                  file=sys.stderr, flush=True)
            runs.append(row)
            torch.cuda.empty_cache()
    return {"cost": cost, "cost_workload": f"rms Mach 1 beta 100 turbulence {n}^3, {a.steps} steps",
            "robustness": runs, "max_steps": a.abl_steps}


def config2_form(a, wombat, inputs):
    """Decaying subsonic MHD turbulence, 256^3 FP64 (rms Mach 0.5, beta 1e4,
    seed 1002), advanced config2_steps CFL-0.4 steps from its initial state:
    throughput and the invariants (sums of the conserved variables relative
    to the sums of their absolute values; corner div B)."""
    import torch
    n = 256
    u = inputs.turbulence((n, n, n), mach=0.5, beta=1e4, seed=1002, device="cuda")
    ctx = wombat.Context(n, n, n, precision=wombat.WW_FP64, cfl=0.4)
    sl = inputs.interior_slices(n, n, n)
    s0 = ctx.sums(u)
    scale = u[sl].abs().sum(dim=(1, 2, 3)).double().cpu().tolist()
    d0, _ = ctx.divb(u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.config2_steps):
        ctx.step(u, 0.0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s1 = ctx.sums(u)
    d1, _ = ctx.divb(u)
    drift = [abs(x - y) / z for x, y, z in zip(s1, s0, scale)]
    res = {"value": n ** 3 * 4 * a.config2_steps / el, "unit": "zone-stage updates/s", "dtype": "f64",
           "ms_per_step": el / a.config2_steps * 1e3, "steps": a.config2_steps,
           "workload": "decaying MHD turbulence 256^3 periodic, rms Mach 0.5, beta 1e4, seed 1002, FP64, "
                       "CFL 0.4 steps from the initial state (each step's CFL dt read back to the host)",
           "sum_drift_rel_max": max(drift), "corner_divb_max": [d0, d1]}
    print(f"[bench] 256^3 subsonic: {res['value']:.3e} zone-stage/s, sum drift {max(drift):.1e}, "
          f"div B {d0:.1e} -> {d1:.1e}", file=sys.stderr, flush=True)
    del ctx, u
    return res


def cpu_model():
    """Host CPU model from lscpu (model name, family and model numbers, CPU and
    socket counts), else the model name from /proc/cpuinfo."""
    import subprocess
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        f = {}
        for line in txt.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                f.setdefault(k.strip(), v.strip())
        if "Model name" in f:
            extra = [f"{k.lower()} {f[k]}" for k in ("CPU family", "Model") if k in f]
            extra += [f"{f[k]} {k.lower().replace('(s)', 's')}" for k in ("CPU(s)", "Socket(s)") if k in f]
            return f["Model name"] + (" (" + ", ".join(extra) + ")" if extra else "")
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def host_threads():
    """Threads the all-core oracle runs on: OMP_NUM_THREADS if set, else the
    CPUs this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def cpu_baseline(n, n_omp):
    """The FP64 oracle on the host: one full RK4 step (CFL dt + 4 stages) of
    the same turbulence recipe, serial on an n^3 box and with OpenMP (the same
    source, k-planes shared among threads) on all host threads on an n_omp^3
    box: bounded samples of the 512^3 workload."""
    from oracle import oracle
    from paper_1808_10633_amd import inputs

    def run(m, threads):
        got = oracle.set_threads(threads)
        u = inputs.turbulence((m, m, m), mach=1.0, beta=100.0, seed=1003).numpy().copy()
        g = oracle.Grid(m, m, m, 1.0 / m, 1.0 / m, 1.0 / m, cfl=0.4)
        t0 = time.perf_counter()
        dt = oracle.cfl_dt(g, u)
        oracle.rk4_step(g, u, dt)
        return m ** 3 * 4 / (time.perf_counter() - t0), time.perf_counter() - t0, got

    v1, t1, _ = run(n, 1)
    threads = host_threads()
    vn, tn, used = run(n_omp, threads)
    oracle.set_threads(1)
    model = cpu_model()
    return {"value": vn, "unit": "zone-stage updates/s", "cores": used, "kind": "oracle",
            "sample": f"one RK4 step (CFL dt + 4 stages) of the {n_omp}^3 box of the same turbulence recipe, "
                      f"C oracle built with OpenMP over k-planes, {used} threads, {tn:.1f} s",
            "cpu_model": model,
            "single_core": {"value": v1, "cores": 1,
                            "sample": f"one RK4 step of the {n}^3 box, serial C oracle, {t1:.1f} s"}}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); the multi-GPU path is a "
              "design (halo-exchanged bricks) that the library does not implement", file=sys.stderr)
        sys.exit(2)
    if a.copy_mib:
        copy_calibration(a.copy_mib)
        return
    import torch

    from paper_1808_10633_amd import inputs, opcount, wombat
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if a.fp32_box:
        print(json.dumps({"fp32_box": fp32_box(a, wombat, inputs, opcount)}), flush=True)
        return
    if a.precision_box:
        print(json.dumps({"precision_box": precision_box(a, wombat, inputs)}), flush=True)
        return
    if a.patch_sweep:
        print(json.dumps({"patch_sweep": patch_sweep(a, wombat, inputs), "unit": "zone-stage updates/s",
                          "dtype": "f32 (f64 islands)", "steps": a.steps}), flush=True)
        return
    if a.ablation:
        print(json.dumps({"ablation": ablation(a, wombat, inputs)}), flush=True)
        return
    n = a.n
    u = inputs.turbulence((n, n, n), mach=1.0, beta=100.0, seed=1003, device="cuda")
    u_ic = u.clone()
    ctx = wombat.Context(n, n, n, precision=wombat.WW_FP64, cfl=0.4)
    print(f"[bench] {n}^3 FP64 turbulence ready; warmup {a.warmup}", file=sys.stderr, flush=True)
    dts = []
    for _ in range(a.warmup):
        dts.append(ctx.step(u, 0.0))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        dts.append(ctx.step(u, 0.0))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    print(f"[bench] {a.steps} steps in {el:.3f} s", file=sys.stderr, flush=True)
    zs = n ** 3 * 4 * a.steps / el
    ms_step = el / a.steps * 1e3

    # kernels of a step by HIP events on the library stream; the dominant one
    # (longest per step) carries the roofline
    ms = ctx.time_kernels(u, reps=a.reps)
    roof, roofs = rooflines(ms, n, "fp64", opcount, FP64_VECTOR_PEAK_TFLOPS)
    out = {"metric": METRIC, "value": zs, "unit": "zone-stage updates/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"decaying MHD turbulence {n}^3 periodic, rms Mach 1.0, beta 100, "
                                  "gamma 5/3, FP64 characteristic WENO5 + CT + RK4, CFL 0.4 step",
                      "n": n, "precision": "fp64"},
           "roofline": roof, "rooflines": roofs, "kernels": kernel_table(ms, ms_step)}
    # the FP64 reference of the precision form continues, untimed, to the
    # compared step count (the timed window is unchanged)
    while len(dts) < a.compare_steps:
        dts.append(ctx.step(u, 0.0))
    torch.cuda.synchronize()
    del ctx
    torch.cuda.empty_cache()

    if not a.no_fp32:
        # precision form: FP32 state/fluxes/weights, FP64 islands; same initial
        # state, the FP64 run's step sizes replayed (its own CFL reduction
        # still runs every step), final states compared after compare_steps
        u32 = u_ic.float().contiguous()
        c32 = wombat.Context(n, n, n, precision=wombat.WW_FP32_MIXED, cfl=0.4)
        for i in range(a.warmup):
            c32.cfl_dt(u32)
            c32.step(u32, dts[i])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(a.steps):
            c32.cfl_dt(u32)
            c32.step(u32, dts[a.warmup + i])
        torch.cuda.synchronize()
        el32 = time.perf_counter() - t0
        ms32 = c32.time_kernels(u32, reps=a.reps)
        for i in range(a.warmup + a.steps, len(dts)):
            c32.cfl_dt(u32)
            c32.step(u32, dts[i])
        torch.cuda.synchronize()
        sl = inputs.interior_slices(n, n, n)
        l1, linf = [], []
        for v in range(8):
            d = (u32[sl][v].double() - u[sl][v]).abs()
            ref = u[sl][v].abs()
            if float(ref.max()) > 0:
                l1.append(float(d.mean() / ref.mean()))
                linf.append(float(d.max() / ref.max()))
        r32, rs32 = rooflines(ms32, n, "fp32", opcount, FP32_VECTOR_PEAK_TFLOPS)
        out["forms"] = {"fp32_mixed": {
            "value": n ** 3 * 4 * a.steps / el32, "ms_per_step": el32 / a.steps * 1e3,
            "speedup_vs_fp64": (n ** 3 * 4 * a.steps / el32) / zs, "dtype": "f32 (f64 islands)",
            "l1_rel_vs_fp64_max_var": max(l1), "linf_rel_vs_fp64_max_var": max(linf),
            "l1_rel_vs_fp64": l1, "linf_rel_vs_fp64": linf,
            "compared_after_steps": len(dts),
            "roofline": r32, "rooflines": rs32, "kernels": kernel_table(ms32, el32 / a.steps * 1e3)}}
        print(f"[bench] fp32 form: L1 {max(l1):.2e}, Linf {max(linf):.2e} after {len(dts)} steps",
              file=sys.stderr, flush=True)
        del c32, u32
        torch.cuda.empty_cache()
    del u, u_ic
    torch.cuda.empty_cache()

    if a.config2_steps > 0:
        out.setdefault("forms", {})["fp64_256_subsonic"] = config2_form(a, wombat, inputs)
        torch.cuda.empty_cache()
    if a.batch_patches > 0:
        out.setdefault("forms", {})["batched_fp32"] = batched_form(a, wombat, inputs, opcount)
        torch.cuda.empty_cache()
    if not a.no_learned:
        from paper_1808_10633_amd import router
        out.setdefault("forms", {})["learned_fp32"] = learned_form(a, wombat, inputs, router)
        torch.cuda.empty_cache()
    if not a.no_cpu:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(a.cpu_n, a.cpu_omp_n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
