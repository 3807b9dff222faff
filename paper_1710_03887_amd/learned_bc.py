"""Learned boundary closure workflow on the trumpet scene.

1. Run the trumpet in an outer box three times larger than the target
   (truncated) box, which contains the truncated mesh element for element,
   and sample, on the faces that form the truncated box's outer boundary,
   the interior trace and the exterior trace (the larger domain's own
   solution) every few steps -- the data the closure learns from.
2. Train the network on those samples (Adam, cosine step-size decay).
3. Run the truncated box with the characteristic ghost and with the learned
   ghost in lockstep with the larger domain (same fixed time step) and
   measure the interior reflection error: the pressure perturbation of the
   truncated run minus the larger run's on the truncated mesh, in a
   volume-weighted nodal L2 norm accumulated over the samples of a run,
   relative to the same norm of the larger run's pressure perturbation.

Every solver and network step runs in libdg.so; torch holds device memory
and does the bookkeeping of samples and norms.
"""
import math
import time

import numpy as np

from . import _lib as dg

P0, RHO0, GAMMA = 1.0 / 1.4, 1.0, 1.4
ALPHA = 2 * math.pi * 565.0 / 343.0
LEVEL_NORM = 0.1 * P0    # fixed scale used to measure a face's amplitude
NORM = 0.0               # the network sees each face scaled by its own largest |q'|


def _torch():
    import torch
    return torch


class Scene:
    """The nested pair of meshes and the truncated box's outer faces."""

    def __init__(self, target_K=8000, scale=3.0):
        from workloads.trumpet import trumpet_nested
        from workloads import BC_OUTFLOW_CHAR
        self.target_K = target_K
        self.big, self.small, self.emap = trumpet_nested(target_K, scale)
        k, f = np.nonzero(self.small["bc"] == BC_OUTFLOW_CHAR)
        self.small_faces = (k, f)
        self.big_faces = self.emap[k] * 4 + f

    def context(self, which, amp, learned=False):
        from workloads import BC_LEARNED, BC_OUTFLOW_CHAR
        m = self.big if which == "big" else self.small
        bc = m["bc"].copy()
        if learned:
            bc[bc == BC_OUTFLOW_CHAR] = BC_LEARNED
        return dg.dg_mesh_setup(m["xyz"], m["EToV"], bc, 4, gamma=GAMMA, rho0=RHO0, p0=P0,
                                inflow_amp=amp, inflow_alpha=ALPHA)


def stable_dt(ctx, cfl=0.45):
    torch = _torch()
    q = torch.zeros((ctx.K, 5, ctx.Np), dtype=torch.float32, device="cuda")
    return dg.dg_stable_dt(ctx, q, cfl)


def sample_run(scene, amp, t_end, every=50, floor=1e-3, dt=None):
    """Run the larger domain at inflow amplitude `amp` (absolute p') and
    return device tensors (X, Y, level) of the samples whose face amplitude
    level = max |rho'| c0^2 is >= floor * amp, plus the fixed dt used (the
    rest-state CFL step with a margin for the flow speed, or `dt`).  Rows
    are scaled per face (NORM = 0)."""
    torch = _torch()
    ctx = scene.context("big", amp)
    dt = dt or stable_dt(ctx)
    nsteps = int(t_end / dt)
    q = torch.zeros((ctx.K, 5, ctx.Np), dtype=torch.float32, device="cuda")
    res = torch.zeros_like(q)
    faces = torch.tensor(scene.big_faces, dtype=torch.int64, device="cuda")
    nf = len(scene.big_faces)
    Xs, Ys, Ls = [], [], []
    t = 0.0
    done = 0
    Xl = torch.empty((nf, 78), dtype=torch.float32, device="cuda")
    while done < nsteps:
        n = min(every, nsteps - done)
        t = dg.dg_run_fixed(ctx, q, res, n, dt, t)
        done += n
        X = torch.empty((nf, 78), dtype=torch.float32, device="cuda")
        Y = torch.empty((nf, 75), dtype=torch.float32, device="cuda")
        dg.dg_sample_traces(ctx, q, faces, LEVEL_NORM, Xl, None)
        dg.dg_sample_traces(ctx, q, faces, NORM, X, Y)
        level = Xl[:, 0:15].abs().amax(dim=1) * LEVEL_NORM   # max |rho'| (c0 = 1)
        keep = level >= floor * amp
        if bool(keep.any()):
            Xs.append(X[keep])
            Ys.append(Y[keep])
            Ls.append(level[keep])
    torch.cuda.synchronize()
    if not Xs:
        return None, None, None, dt
    return torch.cat(Xs), torch.cat(Ys), torch.cat(Ls), dt


def train(X, Y, steps=4000, batch=4096, lr0=1e-3, seed=0, log_every=0):
    """Adam with cosine decay over `steps` minibatches drawn (with a seeded
    generator) from the samples.  Returns the network and the loss trace."""
    torch = _torch()
    from workloads.mlp_init import init_params
    m = dg.dg_mlp_create(init_params(seed).astype(np.float32))
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    trace = []
    for it in range(steps):
        lr = lr0 * 0.5 * (1.0 + math.cos(math.pi * it / steps))
        rows = torch.tensor(rng.integers(0, n, batch), dtype=torch.int64, device="cuda")
        want = log_every and (it % log_every == 0 or it == steps - 1)
        L = dg.dg_mlp_train_step(m, X, Y, lr, rows=rows, want_loss=bool(want))
        if want:
            trace.append((it, L))
    torch.cuda.synchronize()
    return m, trace


def _weights(ctx):
    torch = _torch()
    J = dg.dg_geometry(ctx)["J"]
    return torch.tensor(J, dtype=torch.float32, device="cuda")


def reflection_error(scene, amp, t_end, dt, nets=(), every=100, window=None, blends=None):
    """Interior reflection error of the truncated box against the larger
    domain for the characteristic ghost and for each network in `nets`
    (with the matching entry of `blends`, default 1).  Returns
    ([err_char, err_net...], seconds per step of each truncated run)."""
    torch = _torch()
    big = scene.context("big", amp)
    runs = [scene.context("small", amp)]
    blends = blends or [1.0] * len(nets)
    for net, b in zip(nets, blends):
        c = scene.context("small", amp, learned=True)
        dg.dg_set_learned_bc(c, net, NORM, *window, blend=b)
        runs.append(c)
    nsteps = int(t_end / dt)
    emap = torch.tensor(scene.emap, dtype=torch.int64, device="cuda")
    Jb = _weights(big)
    Js = Jb[emap]
    states = []
    for c in [big] + runs:
        q = torch.zeros((c.K, 5, c.Np), dtype=torch.float32, device="cuda")
        states.append((c, q, torch.zeros_like(q), torch.empty_like(q)))
    num = [0.0] * len(runs)
    den = 0.0
    secs = [0.0] * len(runs)
    done = 0
    t = [0.0] * len(states)
    while done < nsteps:
        n = min(every, nsteps - done)
        for i, (c, q, r, prim) in enumerate(states):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t[i] = dg.dg_run_fixed(c, q, r, n, dt, t[i])
            if i > 0:
                secs[i - 1] += time.perf_counter() - t0
            dg.dg_state_to_prim(c, q, prim)
        done += n
        pb = states[0][3][:, 4, :][emap]
        den += float((Js[:, None] * pb * pb).sum())
        for i in range(len(runs)):
            d = states[i + 1][3][:, 4, :] - pb
            num[i] += float((Js[:, None] * d * d).sum())
        if done % (20 * every) == 0 or done == nsteps:
            print(f"reflection error: step {done}/{nsteps}", flush=True)
    errs = [math.sqrt(x / den) for x in num]
    return errs, [s / nsteps for s in secs]


def layer_sigma(ctx, scale, sigma_max, half=(1.15, 1.0, 1.0), center=(0.65, 0.0, 0.0)):
    """Damping rates [K, Np] (device, library node order) of an absorbing
    layer filling the shell between the small box (half extents `half` about
    `center`) and the outer box `scale` times larger: sigma_max xi^2, xi the
    node's largest normalized depth into the shell over the three axes."""
    torch = _torch()
    x = dg.dg_nodes(ctx)                                      # [K, Np, 3]
    h = np.asarray(half)
    depth = (np.abs(x - np.asarray(center)) - h) / ((scale - 1.0) * h)
    xi = np.clip(depth, 0.0, 1.0).max(axis=-1)
    return torch.tensor(sigma_max * xi * xi, dtype=torch.float32, device="cuda").contiguous()


def outer_domains(scene, amp, t_end, dt, configs, every=100):
    """Interior error on outer boxes `scale` times the small box (each
    containing the small mesh element for element), closed by the
    characteristic ghost, with an absorbing layer of peak rate sigma_max in
    the shell around the small box when sigma_max > 0; measured like
    reflection_error against the scene's larger domain on the small box's
    elements.  configs: [(scale, sigma_max)].  Returns ([error], [seconds per
    step], [elements]) per config."""
    torch = _torch()
    from workloads.trumpet import trumpet_nested
    big = scene.context("big", amp)
    runs, maps, keep = [], [], []
    for sc, smax in configs:
        if sc == 1.0:   # the small box itself (a layer then lies inside it: not a fair comparison)
            if smax > 0:
                raise ValueError("an absorbing layer needs an outer box larger than the small box")
            mid, emap = scene.small, np.arange(len(scene.small["EToV"]))
        else:
            mid, small, emap = trumpet_nested(scene.target_K, sc)
            assert np.array_equal(small["EToV"], scene.small["EToV"])
        c = dg.dg_mesh_setup(mid["xyz"], mid["EToV"], mid["bc"], 4, gamma=GAMMA, rho0=RHO0,
                             p0=P0, inflow_amp=amp, inflow_alpha=ALPHA)
        if smax > 0:
            sig = layer_sigma(c, sc, smax)
            dg.dg_set_damping(c, sig)
            keep.append(sig)
        runs.append(c)
        maps.append(torch.tensor(emap, dtype=torch.int64, device="cuda"))
    emap_big = torch.tensor(scene.emap, dtype=torch.int64, device="cuda")
    Js = _weights(big)[emap_big]
    states = []
    for c in [big] + runs:
        q = torch.zeros((c.K, 5, c.Np), dtype=torch.float32, device="cuda")
        states.append((c, q, torch.zeros_like(q), torch.empty_like(q)))
    num, den, secs = [0.0] * len(runs), 0.0, [0.0] * len(runs)
    t = [0.0] * len(states)
    nsteps, done = int(t_end / dt), 0
    while done < nsteps:
        n = min(every, nsteps - done)
        for i, (c, q, r, prim) in enumerate(states):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t[i] = dg.dg_run_fixed(c, q, r, n, dt, t[i])
            if i > 0:
                secs[i - 1] += time.perf_counter() - t0
            dg.dg_state_to_prim(c, q, prim)
        done += n
        pb = states[0][3][:, 4, :][emap_big]
        den += float((Js[:, None] * pb * pb).sum())
        for i in range(len(runs)):
            d = states[i + 1][3][:, 4, :][maps[i]] - pb
            num[i] += float((Js[:, None] * d * d).sum())
        if done % (20 * every) == 0 or done == nsteps:
            print(f"outer domains: step {done}/{nsteps}", flush=True)
    return ([math.sqrt(x / den) for x in num], [s_ / nsteps for s_ in secs],
            [c.K for c in runs])


def char_domains(scene, amp, t_end, dt, scales, every=100):
    """outer_domains with the characteristic ghost alone on each box."""
    return outer_domains(scene, amp, t_end, dt, [(sc, 0.0) for sc in scales], every)


def choose_blend(scene, net, window, amp, t_end, dt, blends=(0.25, 0.5, 0.75, 1.0)):
    """The blend weight with the smallest interior reflection error at a
    validation amplitude.  Returns (blend, {blend: error}, char error)."""
    errs, _ = reflection_error(scene, amp, t_end, dt, nets=[net] * len(blends), window=window,
                               blends=list(blends))
    table = dict(zip(blends, errs[1:]))
    return min(table, key=table.get), table, errs[0]


def window_of(levels, factor=2.0):
    """[lo, hi] of the samples' face amplitudes max |p'| (acoustic estimate
    c0^2 |rho'|), widened by `factor` on both sides: where the network is
    used."""
    return float(levels.min()) / factor, float(levels.max()) * factor


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="learned closure: sample, train, evaluate")
    ap.add_argument("--target", type=int, default=50_000, help="truncated box tetrahedra")
    ap.add_argument("--t-end", type=float, default=3.2)
    ap.add_argument("--train-amps", default="0.001,0.002,0.005,0.01,0.02,0.03",
                    help="inflow amplitudes / p0 of the sampling runs")
    ap.add_argument("--eval-amps", default="0.003,0.015")
    ap.add_argument("--val-amp", type=float, default=0.007, help="amplitude / p0 that picks the blend")
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--char-scales", default="1.25,1.5,2.0",
                    help="outer boxes (x the small box) run with the characteristic ghost")
    ap.add_argument("--layers", default="",
                    help="absorbing-layer runs scale:sigma_max,... (shell between the small box "
                         "and the outer box)")
    ap.add_argument("--domains-only", action="store_true",
                    help="skip the learned closure: only the outer-box and layer runs at the "
                         "last evaluation amplitude")
    args = ap.parse_args()
    torch = _torch()
    t0 = time.perf_counter()
    scene = Scene(args.target)
    if args.domains_only:
        a = float(args.eval_amps.split(",")[-1])
        dt = stable_dt(scene.context("big", a * P0))
        configs = [(1.0, 0.0)] + [(float(x), 0.0) for x in args.char_scales.split(",") if x]
        configs += [tuple(float(v) for v in x.split(":")) for x in args.layers.split(",") if x]
        errs, secs, Ks = outer_domains(scene, a * P0, args.t_end, dt, configs)
        rows = [{"scale": sc, "sigma_max": sm, "K": K, "err": e, "s_per_step": t_}
                for (sc, sm), e, t_, K in zip(configs, errs, secs, Ks)]
        print(json.dumps({"amp": a, "dt": dt, "domains": rows}), flush=True)
        return
    Xs, Ys, Ls, dt = [], [], [], None
    for a in [float(x) for x in args.train_amps.split(",")]:
        X, Y, L, dt = sample_run(scene, a * P0, args.t_end, dt=dt)
        if X is not None:
            Xs.append(X)
            Ys.append(Y)
            Ls.append(L)
        print(f"sampled amp {a}: {0 if X is None else X.shape[0]} rows", flush=True)
    X, Y = torch.cat(Xs), torch.cat(Ys)
    win = window_of(torch.cat(Ls))
    t1 = time.perf_counter()
    net, trace = train(X, Y, steps=args.steps, log_every=500)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print("loss", trace, flush=True)
    out = {"target_K": args.target, "K_small": len(scene.small["EToV"]),
           "K_big": len(scene.big["EToV"]), "dt": dt, "rows": int(X.shape[0]),
           "window": win, "train_s": t2 - t1, "sample_s": t1 - t0, "loss": trace, "eval": []}
    blend, table, _ = choose_blend(scene, net, win, args.val_amp * P0, args.t_end, dt)
    out["blend"], out["blend_table"] = blend, table
    print("blend", blend, table, flush=True)
    for a in [float(x) for x in args.eval_amps.split(",")]:
        errs, secs = reflection_error(scene, a * P0, args.t_end, dt, nets=[net], window=win,
                                      blends=[blend])
        out["eval"].append({"amp": a, "err_char": errs[0], "err_learned": errs[1],
                            "gain": errs[0] / errs[1], "s_per_step_char": secs[0],
                            "s_per_step_learned": secs[1]})
        print(json.dumps(out["eval"][-1]), flush=True)
    scales = [float(x) for x in args.char_scales.split(",") if x]
    if scales:
        a = float(args.eval_amps.split(",")[-1])
        errs, secs, Ks = char_domains(scene, a * P0, args.t_end, dt, scales)
        learned = out["eval"][-1]
        rows = [{"scale": 1.0, "K": out["K_small"], "err_char": learned["err_char"],
                 "s_per_step": learned["s_per_step_char"]}]
        rows += [{"scale": sc, "K": K, "err_char": e, "s_per_step": t_}
                 for sc, e, t_, K in zip(scales, errs, secs, Ks)]
        out["char_domains"] = rows
        meet = [r for r in rows if r["err_char"] <= learned["err_learned"]]
        if meet:
            r = min(meet, key=lambda r: r["scale"])
            # DOF-stage updates/s the learned run delivers, counted as the
            # DOFs the characteristic ghost needs for the same error
            out["learned_equivalent_speedup"] = r["s_per_step"] / learned["s_per_step_learned"]
            out["char_scale_needed"] = r["scale"]
        print(json.dumps({"char_domains": rows,
                          "speedup": out.get("learned_equivalent_speedup")}), flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
