"""Throughput of the nodal DG Euler hot path on one MI355X.

Workload (default): the trumpet in a box -- a bore of radius 0.05 joined to
an exponential bell of mouth radius 0.4, inside [-0.5, 1.8] x [-1, 1]^2,
about 200k tetrahedra at order N = 4 (Np = 35), slip walls on the
instrument, the mouthpiece pulse of 0.1 p0 as inflow, characteristic
outflow on the box; fluid initially at rest.  One step is one five-stage
low-storage RK step (five fused stage kernels plus the device-side time-step
reduction), run through dg_run's captured HIP graph with the state resident
in HBM.  value = 5 K Np (DOFs) x 5 stages x steps / wall time.

Prints one JSON line.  Also reports, for the dominant kernel (the fused
stage kernel), its algorithmic HBM bytes per launch over its average
duration timed with HIP events on the stream it runs on, and the FP64 CPU
oracle's rate on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SEGMENTS = 5    # timed steps are split into this many event-timed dg_run calls
RK4A2, RK4B2 = -567301805773.0 / 1357537059087.0, 5161836677717.0 / 13612068292357.0


def geometry_bytes(variant):
    """Geometry bytes per element a stage kernel reads: 9 metric terms and
    4 x (normal, Fscale), FP32 for the tile-cooperative kernel (variant 0),
    FP64 for the role-specialized one."""
    return (9 + 16) * (4 if variant == 0 else 8)


def stage_bytes(K, Np, reads_res=True, variant=0):
    """Algorithmic HBM bytes of one fused stage: state in, residual in/out,
    state out (FP32), geometry (geometry_bytes) and connectivity (4 int32
    neighbours + 4 bytes of face/orientation)."""
    passes = 4 if reads_res else 3
    return K * (passes * 5 * Np * 4 + geometry_bytes(variant) + 4 * 4 + 4)


def kernel_source_hash():
    """Hash of the stage kernel's sources and compile flags."""
    import importlib.util
    h = hashlib.sha256()
    for name in ("csrc/kernels.hip", "csrc/spec_stage.hip", "csrc/physics.hpp", "csrc/kernels.hpp"):
        with open(os.path.join(ROOT, "paper_1710_03887_amd", name), "rb") as f:
            h.update(f.read())
    spec = importlib.util.spec_from_file_location(
        "dg_build", os.path.join(ROOT, "paper_1710_03887_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    h.update(" ".join(mod.FLAGS).encode())
    return h.hexdigest()[:16]


def measured_traffic(form, K, variant):
    """HBM bytes per stage launch from the committed rocprofv3 counter
    summary, or None when absent or taken on a different kernel source,
    workload size or stage-kernel variant."""
    path = os.path.join(ROOT, "profiles", "stage_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(form)
    except (ValueError, OSError):
        return None
    if (not rec or rec.get("kernel_hash") != kernel_source_hash() or rec.get("K") != K
            or rec.get("variant") != variant):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(seconds_budget=30.0):
    """The FP64 oracle on a bounded sample of the same workload: the same
    trumpet-in-box geometry at ~20k tetrahedra, N = 4, one LSERK step."""
    from threadpoolctl import threadpool_info
    from oracle.operators import RefElement
    from oracle.mesh import Mesh
    from oracle import euler, timestep
    from workloads import trumpet_domain
    m = trumpet_domain("box", 20_000)
    ref = RefElement(4)
    mesh = Mesh(ref, m["xyz"], m["EToV"], m["bc"])
    phys = euler.Physics(amp=0.1 / 1.4, alpha=2 * np.pi * 565.0 / 343.0)
    q = np.broadcast_to(phys.q0[None, :, None], (mesh.K, 5, ref.Np)).copy()
    dt = timestep.stable_dt(mesh, q, phys, 0.5)
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    # the oracle's contractions are small matrix products and its gathers are
    # NumPy indexing: it runs at the same rate on one thread as on the whole
    # BLAS pool, so the baseline is taken on one thread (cores = 1), with a
    # shorter run on the full pool beside it
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        stages = 0
        while True:
            q, _ = timestep.lserk_step(lambda y, t: euler.rhs(mesh, y, t, phys), q, 0.0, dt)
            stages += 5
            if time.perf_counter() - t0 > seconds_budget / 3:
                break
        el = time.perf_counter() - t0
    t1 = time.perf_counter()
    for _ in range(2):
        euler.rhs(mesh, q, 0.0, phys)
    el1 = time.perf_counter() - t1
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    out = {"value": 5 * mesh.K * ref.Np * stages / el, "unit": "DOF-stage updates/s",
           "cores": 1, "kind": "oracle",
           "sample": f"trumpet-in-box {mesh.K} tets, N=4, {stages // 5} LSERK step(s) "
                     f"({stages} RHS evaluations) in {el:.1f} s, FP64 NumPy on one thread, "
                     f"host cores={os.cpu_count()}, CPU {model or 'unknown'}"}
    pool = {"value": 5 * mesh.K * ref.Np * 2 / el1, "unit": "DOF-stage updates/s",
            "threads": int(threads),
            "sample": f"2 RHS evaluations of the same sample in {el1:.1f} s on {threads} BLAS threads"}
    return out, pool


def time_single(dg, torch, m, N, form, steps, warmup, kernel_iters):
    """One solve on mesh m: timed dg_run plus the stage kernel timed alone."""
    amp, alpha, p0 = 0.1 / 1.4, 2 * np.pi * 565.0 / 343.0, 1.0 / 1.4
    ctx = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], N, gamma=1.4, rho0=1.0, p0=p0,
                           inflow_amp=amp, inflow_alpha=alpha,
                           precision={"fp32": dg.DG_FP32, "bf16": dg.DG_SPLIT_BF16}[form])
    K, Np = ctx.K, ctx.Np
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    q = torch.zeros((K, 5, Np), dtype=torch.float32, device=dev)   # fluid at rest
    res = torch.zeros_like(q)
    bpc = dg.dg_autotune(ctx, q, res, None, stream=stream)

    t, _ = dg.dg_run(ctx, q, res, warmup, 0.5, 0.0, stream=stream)
    torch.cuda.synchronize()
    # exactly `steps` timed steps, as SEGMENTS back-to-back dg_run calls each
    # bracketed by HIP events on the stream they run on
    seg = [steps // SEGMENTS + (1 if i < steps % SEGMENTS else 0) for i in range(SEGMENTS)]
    seg = [n for n in seg if n > 0]
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in seg]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_end, dt_last = t, 0.0
    for (e0, e1), n in zip(ev, seg):
        e0.record(stream)
        t_end, dt_last = dg.dg_run(ctx, q, res, n, 0.5, t_end, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    seg_ms = [e0.elapsed_time(e1) for e0, e1 in ev]
    ms = sum(seg_ms)
    dof = 5 * K * Np
    seg_rate = [dof * 5 * n / (x * 1e-3) for n, x in zip(seg, seg_ms)]

    # dominant kernel: the fused stage, timed alone on the same stream,
    # SEGMENTS batches of kernel_iters launches (median reported)
    qb = torch.empty_like(q)
    for _ in range(3):
        dg.dg_stage(ctx, q, qb, res, RK4A2, RK4B2, t_end, dt_last, stream=stream)
    batches = []
    for _ in range(SEGMENTS):
        k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        k0.record(stream)
        for i in range(kernel_iters):
            src, dst = (q, qb) if i % 2 == 0 else (qb, q)
            dg.dg_stage(ctx, src, dst, res, RK4A2, RK4B2, t_end, dt_last, stream=stream)
        k1.record(stream)
        torch.cuda.synchronize()
        batches.append(k0.elapsed_time(k1) * 1e-3 / kernel_iters)
    kernel_s = float(np.median(batches))
    # dg_rhs alone (q in, rhs out, geometry and connectivity: 40 Np + 120
    # algorithmic bytes per element with the tile-cooperative kernel)
    r = torch.empty_like(q)
    r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    r0.record(stream)
    for _ in range(kernel_iters):
        dg.dg_rhs(ctx, q, r, t_end, stream=stream)
    r1.record(stream)
    torch.cuda.synchronize()
    rhs_s = r0.elapsed_time(r1) * 1e-3 / kernel_iters
    variant = dg.dg_get_kernel(ctx)
    rhs_bytes = K * (40 * Np + geometry_bytes(variant) + 20)
    nbytes = stage_bytes(K, Np, True, variant)
    return {"K": K, "N": N, "Np": Np, "dof": dof, "ms": ms, "wall_s": wall, "t_end": t_end,
            "dt_last": dt_last, "value": dof * 5 * steps / (ms * 1e-3), "kernel_s": kernel_s,
            "segments": {"steps": seg, "ms": seg_ms, "median_value": float(np.median(seg_rate)),
                         "min_value": min(seg_rate), "max_value": max(seg_rate),
                         "spread": (max(seg_rate) - min(seg_rate)) / float(np.median(seg_rate))},
            "kernel_batches_ms": [b * 1e3 for b in batches],
            "bytes": nbytes, "achieved": nbytes / kernel_s / 1e9, "blocks_per_cu": bpc,
            "kernel_variant": variant,
            "rhs_ms": rhs_s * 1e3, "rhs_GBs": rhs_bytes / rhs_s / 1e9, "rhs_bytes": rhs_bytes,
            "kernel": ("stage_kernel" if variant == 0 else "spec_stage_kernel") +
                      f"<{N},MODE_STAGE>"}


def stage_only(dg, torch, m, N, form, launches):
    """Launches of the fused stage kernel alone on a small random state
    (for profiler counters): no autotuning, no other kernels in between."""
    ctx = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], N, gamma=1.4, rho0=1.0, p0=1.0 / 1.4,
                           inflow_amp=0.1 / 1.4, inflow_alpha=2 * np.pi * 565.0 / 343.0,
                           precision={"fp32": dg.DG_FP32, "bf16": dg.DG_SPLIT_BF16}[form])
    dev = torch.device("cuda", 0)
    g = torch.Generator(device="cpu").manual_seed(0)
    q = (1e-3 * torch.randn((ctx.K, 5, ctx.Np), generator=g)).to(dev)
    res, qb = torch.zeros_like(q), torch.empty_like(q)
    for i in range(launches):
        src, dst = (q, qb) if i % 2 == 0 else (qb, q)
        dg.dg_stage(ctx, src, dst, res, RK4A2, RK4B2, 0.1, 1e-5)
    torch.cuda.synchronize()
    print(json.dumps({"stage_only": launches, "K": ctx.K, "N": N, "form": form,
                      "kernel_variant": dg.dg_get_kernel(ctx)}), flush=True)


def batch_stage_bytes(Ks, Np, members=16):
    """Algorithmic HBM bytes of one batched stage: four FP32 state passes
    per member-innermost DOF plus each element's geometry and connectivity
    read once for all members."""
    return sum(K * (4 * 5 * Np * members * 4 + (9 + 16) * 8 + 4 * 4 + 4) for K in Ks)


def time_batch(dg, torch, steps, warmup, kernel_iters, scale=1.0):
    """The ensemble: full box (50k), sphere of radius 1.5 (80k) and half
    domain (30k) around the trumpet, 16 pulse amplitudes log-spaced over
    0.1%-10% of p0 each, N = 3, FP32, launch shape from the autotuner."""
    from workloads import trumpet_domain, locality_order, reorder
    p0, alpha, N = 1.0 / 1.4, 2 * np.pi * 565.0 / 343.0, 3
    meshes = [trumpet_domain(kind, int(n * scale))
              for kind, n in (("box", 50_000), ("sphere", 80_000), ("half", 30_000))]
    # elements in the Z-order of their centroids (the ensemble's 1 GB of
    # state outgrows the last-level cache)
    meshes = [reorder(m, locality_order(m)) for m in meshes]
    ctxs = [dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], N, gamma=1.4, rho0=1.0, p0=p0,
                             inflow_amp=0.0, inflow_alpha=alpha) for m in meshes]
    Ks, Np = [c.K for c in ctxs], ctxs[0].Np
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    b = dg.dg_batch_create(ctxs, 16)
    q = [torch.zeros((K, 5, Np, 16), dtype=torch.float32, device=dev) for K in Ks]
    res = [torch.zeros_like(x) for x in q]
    amps = p0 * np.logspace(-3, -1, 16)
    bpc, waves = dg.dg_batch_autotune(b, q, res, None, stream=stream)
    t = dg.dg_batch_run(b, q, res, amps, warmup, 0.5, None, stream=stream)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    t = dg.dg_batch_run(b, q, res, amps, steps, 0.5, t, stream=stream)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    dof = 5 * Np * 16 * sum(Ks)
    # per-stage average over whole steps (the two one-block scalar kernels of
    # each step and one start-of-run rate pass included)
    k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    k0.record(stream)
    t = dg.dg_batch_run(b, q, res, amps, kernel_iters, 0.5, t, stream=stream)
    k1.record(stream)
    torch.cuda.synchronize()
    step_s = k0.elapsed_time(k1) * 1e-3 / kernel_iters
    nbytes = batch_stage_bytes(Ks, Np)
    return {"K": Ks, "N": N, "Np": Np, "members": 16, "dof": dof, "ms": ms,
            "value": dof * 5 * steps / (ms * 1e-3), "ms_per_step": ms / steps,
            "blocks_per_cu": bpc, "waves_per_block": waves, "bytes_per_stage": nbytes,
            "stage_ms_step_avg": step_s / 5 * 1e3,
            "achieved_GBs_step_avg": nbytes * 5 / step_s / 1e9,
            "frac_step_avg": nbytes * 5 / step_s / 1e9 / HBM_PEAK_GBS,
            "t_min": float(t.min()), "t_max": float(t.max())}


def time_precision_n5(dg, torch, steps):
    """The precision workload: the trumpet in the box at 1,165,248 tets,
    N = 5, FP32 and split-BF16 forms, each with its autotuned launch.  Its
    elements are put in the Z-order of their centroids: the state (1.3 GB)
    outgrows the last-level cache, and neighbour traces then come from HBM
    unless neighbours lie close in memory."""
    from workloads import trumpet_domain, locality_order, reorder
    m = trumpet_domain("box", 1_200_000)
    m = reorder(m, locality_order(m))
    out = {}
    for form in ("fp32", "bf16"):
        o = time_single(dg, torch, m, 5, form, steps, 5, 10)
        out[form] = {"value": o["value"], "ms_per_step": o["ms"] / steps,
                     "stage_kernel_ms": o["kernel_s"] * 1e3, "stage_GBs": o["achieved"],
                     "frac": o["achieved"] / HBM_PEAK_GBS, "kernel": o["kernel"],
                     "blocks_per_cu": o["blocks_per_cu"]}
        torch.cuda.empty_cache()
    out["K"], out["N"], out["steps"] = o["K"], 5, steps
    out["bf16_speedup"] = out["bf16"]["value"] / out["fp32"]["value"]
    return out


# stand-ins for the paper's sensors (Section 3, Table 2) placed by their
# relation to the bell plane (x = 1) and to the outer boundary of this box
# (x = 1.8, y = 1), a hair off the z = 0 mesh plane: 1 cm in front of the bell
# edge near the top wall, 2 cm and 1 cm before the far wall on the axis,
# midway up in front of the bell, and inside the bore near the mouthpiece
SENSORS = ((1.01, 0.99, 0.003), (1.78, 0.0, 0.003), (1.79, 0.0, 0.003), (1.29, 0.57, 0.003),
           (0.01, 0.0, 0.003))


def time_probes(dg, torch, m, steps=200):
    """Recording the sensors every step on the c2 trumpet (fixed dt) against
    the same run without recording, and the spectra of the recorded series."""
    amp, alpha, p0 = 0.1 / 1.4, 2 * np.pi * 565.0 / 343.0, 1.0 / 1.4
    ctx = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], 4, gamma=1.4, rho0=1.0, p0=p0,
                           inflow_amp=amp, inflow_alpha=alpha)
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    q = torch.zeros((ctx.K, 5, ctx.Np), dtype=torch.float32, device=dev)
    res = torch.zeros_like(q)
    dg.dg_autotune(ctx, q, res, None, stream=stream)
    dg.dg_probe_setup(ctx, SENSORS)
    dt = dg.dg_stable_dt(ctx, q, 0.5, stream=stream)
    series = torch.empty((steps, len(SENSORS)), dtype=torch.float32, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    dg.dg_run_fixed(ctx, q, res, 4, dt, 0.0, stream=stream)
    dg.dg_run_probes(ctx, q, res, 4, dt, 0.0, series[:4], stream=stream)
    q.zero_(); res.zero_()
    ev[0].record(stream)
    t = dg.dg_run_fixed(ctx, q, res, steps, dt, 0.0, stream=stream)
    ev[1].record(stream)
    q.zero_(); res.zero_()
    ev[2].record(stream)
    t = dg.dg_run_probes(ctx, q, res, steps, dt, 0.0, series, stream=stream)
    ev[3].record(stream)
    db = torch.empty((len(SENSORS), steps // 2 + 1), dtype=torch.float32, device=dev)
    ev[4].record(stream)
    # dB re 20 micropascal, with p0 standing for one atmosphere (101,325 Pa)
    dg.dg_spectrum(series, 2e-5 / 101325.0 * p0, db, stream=stream)
    ev[5].record(stream)
    torch.cuda.synchronize()
    plain, rec = ev[0].elapsed_time(ev[1]) / steps, ev[2].elapsed_time(ev[3]) / steps
    return {"K": ctx.K, "N": 4, "sensors": len(SENSORS), "steps": steps, "dt": dt, "t_end": t,
            "ms_per_step_plain": plain, "ms_per_step_recording": rec,
            "recording_overhead": rec / plain - 1.0, "spectrum_ms": ev[4].elapsed_time(ev[5]),
            "max_abs_p_prime": float(series.abs().max())}


def time_quadrature(dg, torch, m, steps=200):
    """The paper's own discretization (weak form with Gauss quadrature, RK2)
    on the c2 trumpet at N = 1 (the order the paper ran) and N = 2: dg_run
    throughput and the per-stage kernel time (a step is two stages)."""
    amp, alpha, p0 = 0.1 / 1.4, 2 * np.pi * 565.0 / 343.0, 1.0 / 1.4
    out = {}
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    for N in (1, 2):
        ctx = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], N, gamma=1.4, rho0=1.0, p0=p0,
                               inflow_amp=amp, inflow_alpha=alpha, quadrature=True)
        K, Np = ctx.K, ctx.Np
        q = torch.zeros((K, 5, Np), dtype=torch.float32, device=dev)
        res = torch.zeros_like(q)
        t, _ = dg.dg_run(ctx, q, res, 10, 0.3, 0.0, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        t, dt_last = dg.dg_run(ctx, q, res, steps, 0.3, t, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        # stage kernel alone: one right-hand side per launch in MODE_RHS
        r = torch.empty_like(q)
        k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(3):
            dg.dg_rhs(ctx, q, r, t, stream=stream)
        k0.record(stream)
        for _ in range(20):
            dg.dg_rhs(ctx, q, r, t, stream=stream)
        k1.record(stream)
        torch.cuda.synchronize()
        rhs_ms = k0.elapsed_time(k1) / 20
        # an RK2 stage moves on average 2.5 FP32 state passes plus geometry
        nbytes = K * (50 * Np + 220)
        out[f"N{N}"] = {"K": K, "Np": Np, "steps": steps, "ms_per_step": ms / steps,
                        "value": 5 * K * Np * 2 * steps / (ms * 1e-3), "dt_last": dt_last,
                        "rhs_kernel_ms": rhs_ms,
                        "stage_GBs": nbytes / (ms / steps / 2 * 1e-3) / 1e9}
        dg.dg_destroy(ctx)
    return out


def time_curved(dg, torch, steps=100, target_K=80_000, N=4):
    """The spherical trumpet domain with its outer side faces laid onto the
    sphere (curved isoparametric boundary elements) against the same mesh
    with flat faces: one LSERK stage (stage kernel, plus the curved pass and
    the save of the curved elements' residual) and dg_run steps."""
    from workloads import trumpet_domain
    from workloads.curved import sphere_domain_map, curved_nodes
    amp, alpha, p0 = 0.1 / 1.4, 2 * np.pi * 565.0 / 343.0, 1.0 / 1.4
    m = sphere_domain_map(trumpet_domain("sphere", target_K))
    ctx = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], N, gamma=1.4, rho0=1.0, p0=p0,
                           inflow_amp=amp, inflow_alpha=alpha)
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    K, Np = ctx.K, ctx.Np
    q = torch.zeros((K, 5, Np), dtype=torch.float32, device=dev)
    res = torch.zeros_like(q)
    qb = torch.empty_like(q)
    dg.dg_autotune(ctx, q, res, None, stream=stream)
    x = curved_nodes(m, dg.dg_reference_operators(ctx)["rst"])
    out = {"K": K, "N": N, "steps": steps}
    for label in ("curved", "flat"):
        n = dg.dg_set_curved(ctx, x if label == "curved" else None, stream=stream)
        q.zero_(); res.zero_()
        t, _ = dg.dg_run(ctx, q, res, 10, 0.5, 0.0, stream=stream)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(stream)
        t, dt_last = dg.dg_run(ctx, q, res, steps, 0.5, t, stream=stream)
        ev[1].record(stream)
        ev[2].record(stream)
        for i in range(50):
            src, dst = (q, qb) if i % 2 == 0 else (qb, q)
            dg.dg_stage(ctx, src, dst, res, -0.41789047, 0.37921031, t, 1e-5, stream=stream)
        ev[3].record(stream)
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / steps
        out[label] = {"n_curved": n, "ms_per_step": ms, "value": 5 * K * Np * 5 / (ms * 1e-3),
                      "stage_ms": ev[2].elapsed_time(ev[3]) / 50, "dt_last": dt_last}
    out["stage_overhead"] = out["curved"]["stage_ms"] / out["flat"]["stage_ms"] - 1.0
    out["curved_share"] = out["curved"]["n_curved"] / K
    dg.dg_destroy(ctx)
    return out


def time_learned(dg, torch, target_K=50_000, steps=200):
    """Cost of the learned boundary closure per step: the trumpet in the box
    with the characteristic ghost on its outer faces, and the same mesh with
    those faces tagged learned (network with its initial weights, every face
    inside the window, blend 0.5), both with one fixed dt.  The accuracy side
    (the equivalent speedup) needs the sampling and training workflow and is
    not measured here."""
    from workloads import trumpet_domain, BC_LEARNED, BC_OUTFLOW_CHAR
    from workloads.mlp_init import init_params
    m = trumpet_domain("box", target_K)
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    out = {}
    net = dg.dg_mlp_create(init_params(0), stream=stream)
    for label in ("characteristic", "learned"):
        bc = m["bc"].copy()
        if label == "learned":
            bc[bc == BC_OUTFLOW_CHAR] = BC_LEARNED
        ctx = dg.dg_mesh_setup(m["xyz"], m["EToV"], bc, 4, gamma=1.4, rho0=1.0, p0=1.0 / 1.4,
                               inflow_amp=0.01 / 1.4, inflow_alpha=2 * np.pi * 565.0 / 343.0)
        if label == "learned":
            dg.dg_set_learned_bc(ctx, net, 0.0, 0.0, 1e30, blend=0.5)
            out["learned_faces"] = int(len(dg.dg_learned_faces(ctx)))
        K, Np = ctx.K, ctx.Np
        q = torch.zeros((K, 5, Np), dtype=torch.float32, device=dev)
        res = torch.zeros_like(q)
        dt = 8e-5
        t = dg.dg_run_fixed(ctx, q, res, 20, dt, 0.0, stream=stream)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        dg.dg_run_fixed(ctx, q, res, steps, dt, t, stream=stream)
        ev[1].record(stream)
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / steps
        out[label] = {"K": K, "ms_per_step": ms, "value": 5 * K * Np * 5 / (ms * 1e-3)}
        dg.dg_destroy(ctx)
    dg.dg_mlp_destroy(net)
    out["steps"] = steps
    out["cost_ratio"] = out["learned"]["ms_per_step"] / out["characteristic"]["ms_per_step"]
    return out


def time_mlp(dg, torch, rows=65_536, batch=4096, steps=40):
    """The closure's network (78-128-128-75, GELU): Adam steps on 4,096-row
    minibatches of a 65,536-row synthetic set (the training configuration),
    and BF16 inference on all rows."""
    from workloads.mlp_init import init_params
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    m = dg.dg_mlp_create(init_params(0), stream=stream)
    g = torch.Generator(device="cpu").manual_seed(1)
    X = torch.randn((rows, dg.MLP_IN), generator=g).to(dev)
    Y = torch.randn((rows, dg.MLP_OUT), generator=g).to(dev)
    idx = torch.randint(0, rows, (batch,), generator=g).to(dev)
    Yo = torch.empty_like(Y)
    for _ in range(3):
        dg.dg_mlp_train_step(m, X, Y, 1e-3, rows=idx, want_loss=False, stream=stream)
        dg.dg_mlp_infer(m, X, Yo, bf16=True, stream=stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record(stream)
    for _ in range(steps):
        dg.dg_mlp_train_step(m, X, Y, 1e-3, rows=idx, want_loss=False, stream=stream)
    ev[1].record(stream)
    ev[2].record(stream)
    for _ in range(10):
        dg.dg_mlp_infer(m, X, Yo, bf16=True, stream=stream)
    ev[3].record(stream)
    torch.cuda.synchronize()
    dg.dg_mlp_destroy(m)
    step_ms = ev[0].elapsed_time(ev[1]) / steps
    infer_ms = ev[2].elapsed_time(ev[3]) / 10
    flop_row = 2 * (78 * 128 + 128 * 128 + 128 * 75)          # forward multiply-adds x 2
    return {"batch": batch, "train_step_ms": step_ms,
            "train_TFLOPs": 3 * flop_row * batch / (step_ms * 1e-3) / 1e12,
            "infer_rows": rows, "infer_ms": infer_ms,
            "infer_TFLOPs": flop_row * rows / (infer_ms * 1e-3) / 1e12}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--elements", type=int, default=200_000, help="target tetrahedra")
    ap.add_argument("--order", type=int, default=4)
    ap.add_argument("--form", choices=("fp32", "bf16"), default="fp32",
                    help="form of the headline measurement")
    ap.add_argument("--also", default="bf16,batch,n5,probes,quadrature,curved,mlp,learned",
                    help="comma list of extra measurements: bf16, fp32, batch, n5, probes, "
                         "quadrature, curved, mlp, learned (or empty)")
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--n5-steps", type=int, default=100,
                    help="steps per form of the 1.17M-tet N = 5 precision workload")
    ap.add_argument("--kernel-iters", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--stage-only", type=int, default=0, metavar="LAUNCHES",
                    help="counter-collection mode: set up the workload and launch only the "
                         "fused stage kernel this many times (default launch shape), then exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the element-partitioned multi-GPU path "
              "(per-stage face-trace exchange) is designed but not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1710_03887_amd as dg
    from workloads import trumpet_domain

    m = trumpet_domain("box", args.elements)
    N = args.order
    if args.stage_only:
        stage_only(dg, torch, m, N, args.form, args.stage_only)
        return
    r = time_single(dg, torch, m, N, args.form, args.steps, args.warmup, args.kernel_iters)
    K, Np = r["K"], r["Np"]
    traffic = measured_traffic(args.form, K, r["kernel_variant"])
    extra = {}
    for name in [x for x in args.also.split(",") if x]:
        if name in ("fp32", "bf16") and name != args.form:
            o = time_single(dg, torch, m, N, name, args.steps, args.warmup, args.kernel_iters)
            extra[name] = {"value": o["value"], "ms_per_step": o["ms"] / args.steps,
                           "kernel": o["kernel"],
                           "speedup_vs_headline": o["value"] / r["value"],
                           "stage_kernel_ms": o["kernel_s"] * 1e3,
                           "stage_GBs": o["achieved"], "frac": o["achieved"] / HBM_PEAK_GBS,
                           "traffic": measured_traffic(name, K, o["kernel_variant"])}
        elif name == "batch":
            extra["batch"] = time_batch(dg, torch, args.batch_steps, 4, 10)
        elif name == "n5":
            extra["n5"] = time_precision_n5(dg, torch, args.n5_steps)
        elif name == "probes":
            extra["probes"] = time_probes(dg, torch, m)
        elif name == "quadrature":
            extra["quadrature"] = time_quadrature(dg, torch, m)
        elif name == "curved":
            extra["curved"] = time_curved(dg, torch)
        elif name == "mlp":
            extra["mlp"] = time_mlp(dg, torch)
        elif name == "learned":
            extra["learned"] = time_learned(dg, torch)
    if args.copy_mb:
        n = args.copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()

    out = {
        "metric": "DOF-stage updates/s",
        "value": r["value"],
        "unit": "DOF-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"trumpet-in-box, {K} tets, N={N} (Np={Np}), {args.form} form, "
                               "inflow pulse 0.1 p0, characteristic outflow, slip walls",
                   "K": K, "N": N, "Np": Np, "dof": r["dof"], "form": args.form,
                   "t_end": r["t_end"], "dt_last": r["dt_last"], "wall_s": r["wall_s"],
                   "blocks_per_cu": r["blocks_per_cu"], "kernel_variant": r["kernel_variant"],
                   "segments": r["segments"]},
        "roofline": {"bound": "hbm", "achieved": r["achieved"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": r["achieved"] / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, "
                                     "copy-calibrated)",
                     "kernel": r["kernel"], "kernel_ms": r["kernel_s"] * 1e3,
                     "kernel_ms_batches": r["kernel_batches_ms"],
                     "bytes_per_launch": r["bytes"],
                     "dg_rhs": {"ms": r["rhs_ms"], "achieved": r["rhs_GBs"],
                                "frac": r["rhs_GBs"] / HBM_PEAK_GBS,
                                "bytes_per_launch": r["rhs_bytes"]}},
        "forms": extra,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["forms"]["oracle_blas_pool"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
