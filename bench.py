"""Throughput of the locally entropy-stable relaxation RK hot path on one GPU.

Workload: 3-D compressible Euler Taylor-Green vortex, Mach 0.1, periodic
[0, 2 pi]^3, 16^3 elements of degree 3 (262,144 Lobatto nodes, 5 fields),
entropy-conservative flux differencing with local Lax-Friedrichs interfaces,
RK(4,4) at CFL 0.5 with local relaxation every step.  One timed "step" is one
whole locally relaxed RK(4,4) step (4 right-hand sides + stage updates, the
per-element relaxation solve, the global gamma and the relaxed update), with
the CFL step size computed on the device.

Metric: DOF-stage updates per second = nodes x RK stages / time of the step
loop (inputs resident in HBM; no host synchronization inside the loop).  The
K timed steps are replayed from one HIP graph recorded by esrk_run_graph (HIP
events on its stream, device synchronization on both sides); the same K steps
launched eagerly, one esrk_step call each, are reported beside them.  The
headline value is the FP64 path; the FP32-flux / FP64-relaxation path is
reported beside it.  The CPU baseline is the FP64 oracle on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NEL, DEG, MACH = 16, 3, 0.1
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6

# Algorithmic FP64 work of one launch of the fused stage kernel (3-D):
# 90 flop per unordered volume node pair, 130 flop per interface node pair,
# 80 flop per node (primitives, logarithms, entropy variables, stage update).
FLOP_PAIR, FLOP_FACE, FLOP_NODE = 90.0, 130.0, 80.0
# Algorithmic HBM bytes of one middle-stage launch per node (FP64, 5 fields):
# read y, u_old, du; write du, y_next.
BYTES_NODE_STAGE = 5 * 5 * 8

# Measured HBM traffic of that launch (rocprofv3 FETCH_SIZE + WRITE_SIZE,
# calibrated on a copy kernel) and the hash of the stage-kernel sources it was
# taken on; the figure is reported only while those sources are unchanged.
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "rhs_kernel_tgv16_p3_traffic.md")
STAGE_SOURCES = ("paper_2003_08831_amd/csrc/rhs.hip", "paper_2003_08831_amd/csrc/device_math.h",
                 "paper_2003_08831_amd/csrc/internal.h")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-steps", type=int, default=3)
    p.add_argument("--kernel-reps", type=int, default=50)
    p.add_argument("--copy-calib", action="store_true",
                   help="run one 256 MiB device copy kernel first (counter calibration)")
    p.add_argument("--no-variants", action="store_true",
                   help="skip the Navier-Stokes, batched and learned-guess measurements")
    return p.parse_args()


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def ns_variant(esrk, I, torch, precision, steps, warmup, nel=32, deg=4):
    """3-D Navier-Stokes TGV (Re 1600, Pr 0.72, Mach 0.1), whole locally relaxed
    RK(4,4) steps; FP32 mode runs the viscous derivative applies on MFMA."""
    ms = I.tgv_mesh(nel, deg, mu=1.0 / 1600.0)
    cfg = esrk.make_config(ms.dim, ms.deg, ms.nel, ms.lo, ms.hi, gas_gamma=ms.gas_gamma,
                           mu=ms.mu, prandtl=ms.prandtl, precision=precision,
                           tableau=esrk.RK44, cfl=0.5)
    ctx = esrk.Context(cfg)
    u = torch.as_tensor(I.tgv_state(ms, MACH)).to("cuda")
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        ctx.step(u, t)
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    e0.record()
    for _ in range(steps):
        ctx.step(u, t)
    e1.record()
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    rc, bad = ctx.sync_status()
    if rc != 0:
        raise RuntimeError(f"NS variant: device status {esrk.STATUS.get(rc)} at element {bad}")
    N = ctx.N
    del ctx, u
    torch.cuda.empty_cache()
    return {"value": round(N * 4 * steps / (ms_total * 1e-3), 1),
            "ms_per_step": round(ms_total / steps, 4), "nodes": N, "steps": steps}


def batch_variant(esrk, I, torch, steps, nsims=256):
    """256 independent 2-D Euler Kelvin-Helmholtz runs of uneven size (16^2 to
    64^2 elements, p = 3, seeded), FP32 flux, SSPRK(3,3); one kernel per stage
    over all simulations, autotuned tile, steps replayed from a hipGraph."""
    specs = I.kh_batch_specs(nsims, seed=0)
    cfgs, states = [], []
    for nel, amp, k in specs:
        ms = I.kh_mesh(nel, 3)
        cfgs.append(esrk.make_config(2, 3, ms.nel, ms.lo, ms.hi, precision=esrk.FP32_FLUX,
                                     tableau=esrk.SSPRK33, cfl=0.5))
        states.append(I.kh_state(ms, amp, k))
    b = esrk.Batch(cfgs)
    u = torch.zeros(b.len, dtype=torch.float64, device="cuda")
    for s, st in enumerate(states):
        u[b.offsets[s]:b.offsets[s] + st.size] = torch.as_tensor(st, device="cuda")
    t = torch.zeros(b.nsims, dtype=torch.float64, device="cuda")
    g = torch.zeros(b.nsims, dtype=torch.float64, device="cuda")
    tile = b.autotune(u)
    b.step(u, t, g)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        b.run_graph(u, t, steps, g, stream=stream)  # capture + first replay
    stream.synchronize()
    e0, e1 = _events(torch)
    e0.record(stream)
    with torch.cuda.stream(stream):
        b.run_graph(u, t, steps, g, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_graph = e0.elapsed_time(e1)
    e0.record()
    for _ in range(steps):
        b.step(u, t, g)
    e1.record()
    torch.cuda.synchronize()
    ms_eager = e0.elapsed_time(e1)
    rc, bad = b.sync_status()
    if rc != 0:
        raise RuntimeError(f"batch variant: device status {esrk.STATUS.get(rc)} at {bad}")
    N = b.len // 4
    del b, u
    torch.cuda.empty_cache()
    return {"value": round(N * 3 * steps / (ms_graph * 1e-3), 1),
            "ms_per_step": round(ms_graph / steps, 4),
            "eager_ms_per_step": round(ms_eager / steps, 4), "nodes": N, "sims": nsims,
            "tile": tile, "steps": steps}


def mlp_variant(esrk, I, torch, learn, gain_steps=4):
    """Learned first trial point of the relaxation solve on the Navier-Stokes
    TGV (32^3, p = 4): trained on samples logged from Euler TGV (16^3, p = 3)
    and Navier-Stokes TGV steps, then plain / previous-step / network first
    trial points compared on the same increments."""
    runs = []
    ms = I.tgv_mesh(NEL, DEG)
    ctx = esrk.Context(esrk.make_config(3, DEG, ms.nel, ms.lo, ms.hi, tableau=esrk.RK44))
    u = torch.as_tensor(I.tgv_state(ms, MACH)).to("cuda")
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    runs.append(learn.collect(ctx, u, t, 20))
    del ctx, u
    ms = I.tgv_mesh(32, 4, mu=1.0 / 1600.0)
    cfg = esrk.make_config(3, 4, ms.nel, ms.lo, ms.hi, mu=ms.mu, prandtl=ms.prandtl,
                           tableau=esrk.RK44)
    ctx = esrk.Context(cfg)
    u = torch.as_tensor(I.tgv_state(ms, MACH)).to("cuda")
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    runs.append(learn.collect(ctx, u, t, 8))
    model, hist = learn.train(runs, steps=1500, batch=4096, lr=1e-3)
    res = learn.gain(ctx, u, t, gain_steps, model)
    del ctx, u
    torch.cuda.empty_cache()
    return {"samples": hist["n_train"] + hist["n_val"], "train_mse": round(hist["train_final"], 4),
            "val_mse": None if hist["val_final"] is None else round(hist["val_final"], 4),
            "phi_evals_per_elem": {k: round(v["evals"], 3) for k, v in res.items()},
            "relax_ms": {k: round(v["ms"], 4) for k, v in res.items()},
            "max_gamma_diff_vs_plain": {k: v["dgamma"] for k, v in res.items()}}


def run_mode(esrk, I, torch, precision, steps, warmup):
    ms = I.tgv_mesh(NEL, DEG)
    cfg = esrk.make_config(ms.dim, ms.deg, ms.nel, ms.lo, ms.hi, gas_gamma=ms.gas_gamma,
                           precision=precision, tableau=esrk.RK44, cfl=0.5)
    ctx = esrk.Context(cfg)
    u = torch.as_tensor(I.tgv_state(ms, MACH)).to("cuda")
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    stats = torch.zeros(8, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        ctx.step(u, t, 0.0, None, stats)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        ctx.step(u, t, 0.0, None, stats)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = e0.elapsed_time(e1)
    rc, bad = ctx.sync_status()
    if rc != 0:
        raise RuntimeError(f"device status {esrk.STATUS.get(rc)} at element {bad}")
    st = stats.cpu().numpy()
    # the same K steps recorded into one HIP graph (esrk_run_graph) and
    # replayed: the first call records and runs them untimed, the second is
    # timed, with a device synchronization on both sides
    s = torch.cuda.Stream()
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(s):
        ctx.run_graph(u, t, steps, stats, stream=s)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        g0.record(s)
        ctx.run_graph(u, t, steps, stats, stream=s)
        g1.record(s)
    torch.cuda.synchronize()
    rc, bad = ctx.sync_status()
    if rc != 0:
        raise RuntimeError(f"device status {esrk.STATUS.get(rc)} at element {bad}")
    ms_graph = g0.elapsed_time(g1)
    return ctx, u, dict(ms_total=ms_total, ms_graph=ms_graph, wall_s=wall, N=ctx.N,
                        gamma=float(st[0]), dt=float(st[1]), t=float(st[2]))


def relax_modes_variant(esrk, I, torch, steps=10, warmup=2):
    """The headline workload (FP64) with each relaxation of esrk_step: none
    (plain RK(4,4)), local (gamma = min_k gamma_k) and global (one gamma for
    the total entropy; bracket passes driven on the device)."""
    ms = I.tgv_mesh(NEL, DEG)
    cfg = esrk.make_config(ms.dim, ms.deg, ms.nel, ms.lo, ms.hi, gas_gamma=ms.gas_gamma,
                           precision=esrk.FP64, tableau=esrk.RK44, cfl=0.5)
    out = {}
    for name, mode in (("none", esrk.RELAX_NONE), ("local", esrk.RELAX_LOCAL),
                       ("global", esrk.RELAX_GLOBAL)):
        ctx = esrk.Context(cfg)
        ctx.set_relaxation_mode(mode)
        u = torch.as_tensor(I.tgv_state(ms, MACH)).to("cuda")
        t = torch.zeros(1, dtype=torch.float64, device="cuda")
        stats = torch.zeros(8, dtype=torch.float64, device="cuda")
        for _ in range(warmup):
            ctx.step(u, t, 0.0, None, stats)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for _ in range(steps):
            ctx.step(u, t, 0.0, None, stats)
        torch.cuda.synchronize()
        el = time.perf_counter() - w0
        rc, bad = ctx.sync_status()
        if rc != 0:
            raise RuntimeError(f"{name}: device status {esrk.STATUS.get(rc)} at element {bad}")
        out[name] = {"ms_per_step": round(el * 1e3 / steps, 4),
                     "gamma_last": float(stats[0].item())}
        del ctx, u
    return out


def root_methods_variant(esrk, I, torch, steps=10, warmup=2):
    """The headline workload (FP64, local relaxation) with each root-solve
    rule: wall time per step and phi evaluations per active element."""
    ms = I.tgv_mesh(NEL, DEG)
    cfg = esrk.make_config(ms.dim, ms.deg, ms.nel, ms.lo, ms.hi, gas_gamma=ms.gas_gamma,
                           precision=esrk.FP64, tableau=esrk.RK44, cfl=0.5)
    out = {}
    for name, method in (("illinois", esrk.ROOT_ILLINOIS), ("brent", esrk.ROOT_BRENT),
                         ("alefeld", esrk.ROOT_ALEFELD), ("bisection", esrk.ROOT_BISECTION)):
        ctx = esrk.Context(cfg)
        ctx.set_root_method(method)
        u = torch.as_tensor(I.tgv_state(ms, MACH)).to("cuda")
        t = torch.zeros(1, dtype=torch.float64, device="cuda")
        stats = torch.zeros(8, dtype=torch.float64, device="cuda")
        for _ in range(warmup):
            ctx.step(u, t, 0.0, None, stats)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        evals = 0.0
        active = 0.0
        for _ in range(steps):
            ctx.step(u, t, 0.0, None, stats)
        torch.cuda.synchronize()
        el = time.perf_counter() - w0
        st = stats.cpu().numpy()
        active = ctx.ne - st[3]
        evals = st[5] / active if active > 0 else 0.0
        out[name] = {"ms_per_step": round(el * 1e3 / steps, 4),
                     "phi_evals_per_active_elem": round(float(evals), 3),
                     "max_evals": int(st[4])}
        del ctx, u
    return out


def time_stage_kernel(esrk, torch, ctx, u, reps):
    """Average duration of one fused stage-kernel launch (middle RK stage, in
    the configuration esrk_step launches it: phi_k(0) accumulated, no separate
    entropy rate), HIP events on the launch stream (the default stream)."""
    n = u.numel()
    ya = torch.empty(n, dtype=torch.float64, device="cuda")
    du = torch.zeros(n, dtype=torch.float64, device="cuda")
    deta = None
    dt = 1e-3
    ctx.rk_stage(0, dt, u, u, ya, du, deta)
    for _ in range(3):
        ctx.rk_stage(1, dt, u, u, ya, du, deta)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.rk_stage(1, dt, u, u, ya, du, deta)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def measured_traffic():
    """HBM bytes per stage-kernel launch from the committed counter summary,
    or None when it is missing or was taken on other kernel sources."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for s in STAGE_SOURCES:
        with open(os.path.join(ROOT, s), "rb") as f:
            h.update(f.read())
    sha = re.search(r"sha256 over [^`]*`([0-9a-f]{64})`", text)
    tot = re.search(r"\| total HBM bytes per launch \| (\d+) \|", text)
    if not sha or not tot or sha.group(1) != h.hexdigest():
        return None
    return int(tot.group(1))


def cpu_baseline(I, steps):
    import oracle as O
    ms = I.tgv_mesh(NEL, DEG)
    m = O.mesh(ms.dim, ms.deg, ms.nel, ms.lo, ms.hi, gas_gamma=ms.gas_gamma)
    u = I.tgv_state(ms, MACH)
    t = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        r = O.step(m, O.RK44, u, t, cfl=0.5)
        t = r["t"]
    el = time.perf_counter() - t0
    stages = 4 * steps
    return dict(value=ms.N * stages / el, unit="DOF-stage updates/s", cores=1, kind="oracle",
                sample=f"{steps} locally relaxed RK(4,4) steps ({stages} stages) of the "
                       f"16^3 p=3 TGV, {ms.N} nodes, single thread, {el:.1f} s")


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no HIP device visible"}))
        sys.exit(1)
    from paper_2003_08831_amd import esrk
    from paper_2003_08831_amd import inputs as I

    if a.copy_calib:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)  # one elementwise kernel: reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
        del src, dst

    ctx64, u64, r64 = run_mode(esrk, I, torch, esrk.FP64, a.steps, a.warmup)
    ctx32, u32, r32 = run_mode(esrk, I, torch, esrk.FP32_FLUX, a.steps, a.warmup)
    N = r64["N"]
    stages = 4 * a.steps
    # headline: the K steps replayed from one HIP graph; eager launches beside
    val64 = N * stages / (r64["ms_graph"] * 1e-3)
    val32 = N * stages / (r32["ms_graph"] * 1e-3)

    kms = time_stage_kernel(esrk, torch, ctx64, u64, a.kernel_reps)
    ne = ctx64.ne
    n = DEG + 1
    pairs = ne * 3 * n * n * (n * (n - 1) // 2)
    faces = ne * 3 * n * n
    flop = pairs * FLOP_PAIR + faces * FLOP_FACE + N * FLOP_NODE
    tflops = flop / (kms * 1e-3) / 1e12
    gbs = N * BYTES_NODE_STAGE / (kms * 1e-3) / 1e9
    alu_frac = tflops / FP64_VECTOR_PEAK_TFLOPS
    hbm_frac = gbs / HBM_PEAK_GBS
    traffic = measured_traffic()
    if alu_frac >= hbm_frac:
        roof = {"bound": "alu", "achieved": round(tflops, 3), "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(alu_frac, 4), "traffic": traffic}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(hbm_frac, 4), "traffic": traffic}
    roof.update({"kernel": "rhs_kernel<3,4,double> (fused RK stage)",
                 "kernel_ms": round(kms, 4),
                 "traffic_unit": "HBM bytes per launch",
                 "other": {"hbm_GBs": round(gbs, 1), "hbm_frac": round(hbm_frac, 4),
                           "fp64_TFLOPs": round(tflops, 3), "alu_frac": round(alu_frac, 4),
                           "algorithmic_bytes_per_launch": N * BYTES_NODE_STAGE,
                           "traffic_GBs": (round(traffic / (kms * 1e-3) / 1e9, 1)
                                           if traffic else None)}})

    out = {
        "metric": "DOF-stage updates/s incl. local relaxation, FP32-mixed vs FP64, 1 MI355X",
        "value": round(val64, 1),
        "unit": "DOF-stage updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(r64["ms_graph"] / a.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (analytic Taylor-Green initial state)",
        "config": {"workload": "3-D Euler Taylor-Green vortex, Mach 0.1, 16^3 elements, "
                               "degree 3 (262144 nodes), EC flux differencing + LLF, "
                               "RK(4,4) CFL 0.5, local relaxation",
                   "nodes": N, "stages_timed": stages, "precision": "fp64"},
        "eager": {"value": round(N * stages / (r64["ms_total"] * 1e-3), 1),
                  "ms_per_step": round(r64["ms_total"] / a.steps, 4),
                  "fp32_flux_ms_per_step": round(r32["ms_total"] / a.steps, 4),
                  "note": "the same K steps launched one esrk_step call at a time"},
        "fp32_flux": {"value": round(val32, 1), "ms_per_step": round(r32["ms_graph"] / a.steps, 4),
                      "dtype": "f32 flux / f64 relaxation+state", "speedup_vs_fp64":
                      round(val32 / val64, 3)},
        "run": {"gamma_last": r64["gamma"], "dt_last": r64["dt"], "t_end": r64["t"]},
        "roofline": roof,
    }
    if not a.no_variants:
        from paper_2003_08831_amd import learn
        out["variants"] = {
            "ns_tgv_32cubed_p4_fp64": ns_variant(esrk, I, torch, esrk.FP64, 10, 2),
            "ns_tgv_32cubed_p4_fp32_mfma": ns_variant(esrk, I, torch, esrk.FP32_FLUX, 10, 2),
            "kh_batch_256_fp32_graph": batch_variant(esrk, I, torch, 20),
            "learned_guess_ns_tgv": mlp_variant(esrk, I, torch, learn),
            "relaxation_modes_tgv16_p3_fp64": relax_modes_variant(esrk, I, torch),
            "root_methods_tgv16_p3_fp64": root_methods_variant(esrk, I, torch),
        }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(I, a.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
