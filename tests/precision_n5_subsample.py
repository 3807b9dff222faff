"""The precision form at N = 5 against the FP64 oracle on a 19,530-tet
trumpet in the box, 100 steps, pressure pulses of 0.5 %, 2 % and 10 % of p0.

Too slow for the test suite (the oracle needs about 25 CPU minutes per
amplitude), so it runs in two steps:

    python tests/precision_n5_subsample.py oracle <dir>   # CPU, one process per amplitude
    python tests/precision_n5_subsample.py gpu <dir>      # one GPU, reads <dir>

The oracle step stores, per amplitude, the pressure perturbation p - p0 of
its state after 100 steps (FP32 is ample for a 1e-3 comparison) and its
time steps; nothing it stores comes from the library.  The GPU step runs the
FP32 and split-BF16 forms from the same initial state and prints, per form
and amplitude, the mass-matrix relative L2 of p - p_oracle against p_oracle
- p0 (bars: FP32 1e-5, split-BF16 1e-3) and the end time against the
oracle's.

Initial state: a Gaussian pressure pulse of the given amplitude (width 0.2,
in the bell) on the ambient state at rest, with the raised-cosine inflow of
the same amplitude at the mouthpiece, starting a quarter period into the
inflow pulse so that every boundary kind carries signal.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

AMPS = (0.005, 0.02, 0.1)
N = 5
STEPS = 100
CFL = 0.5
TARGET_K = 20_000
ALPHA = 2 * np.pi * 565.0 / 343.0
T0 = 0.25 * 2 * np.pi / ALPHA


def _setup(amp):
    from oracle import euler
    from oracle.mesh import Mesh
    from oracle.operators import RefElement
    from workloads import trumpet_domain, gaussian_pulse
    m = trumpet_domain("box", TARGET_K)
    phys = euler.Physics(amp=amp / 1.4, alpha=ALPHA)
    mesh = Mesh(RefElement(N), m["xyz"], m["EToV"], m["bc"])
    prim = gaussian_pulse(mesh.x, amp * phys.p0, 0.2, (0.85, 0.05, 0.0), phys.rho0, phys.p0,
                          phys.gamma)
    return m, mesh, phys, euler.initial_state(prim, phys.gamma)


def _oracle_one(args):
    amp, out = args
    from oracle import timestep, norms
    _, mesh, phys, q0 = _setup(amp)
    t0 = time.perf_counter()
    q, t, dts = timestep.run(mesh, q0, phys, STEPS, cfl=CFL, t0=T0)
    dp = norms.pressure(q, phys.gamma) - phys.p0
    np.savez(os.path.join(out, f"oracle_amp{amp}.npz"), dp=dp.astype(np.float32), t=t,
             dts=np.array(dts), K=mesh.K)
    return amp, mesh.K, time.perf_counter() - t0


def oracle(out):
    import multiprocessing as mp
    os.makedirs(out, exist_ok=True)
    with mp.get_context("spawn").Pool(len(AMPS)) as pool:
        for amp, K, secs in pool.imap_unordered(_oracle_one, [(a, out) for a in AMPS]):
            print(json.dumps({"amp": amp, "K": K, "oracle_seconds": round(secs, 1)}), flush=True)


def gpu(out):
    import torch
    import paper_1710_03887_amd as dg
    from oracle import norms
    sys.path.insert(0, HERE)
    from helpers import node_perm, phys_kwargs
    rows = []
    for amp in AMPS:
        ref_file = np.load(os.path.join(out, f"oracle_amp{amp}.npz"))
        m, mesh, phys, q0 = _setup(amp)
        assert int(ref_file["K"]) == mesh.K
        for name, prec, bar in (("fp32", dg.DG_FP32, 1e-5), ("split_bf16", dg.DG_SPLIT_BF16, 1e-3)):
            ctx = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], N, precision=prec,
                                   **phys_kwargs(phys))
            perm = node_perm(ctx, mesh.ref)
            qd = torch.tensor((q0 - phys.q0[None, :, None])[:, :, perm], dtype=torch.float32,
                              device="cuda").contiguous()
            res = torch.zeros_like(qd)
            t, _ = dg.dg_run(ctx, qd, res, STEPS, CFL, T0)
            torch.cuda.synchronize()
            x = qd.double().cpu().numpy()
            q = np.empty_like(x)
            q[:, :, perm] = x
            q += phys.q0[None, :, None]
            dp = norms.pressure(q, phys.gamma) - phys.p0
            dref = ref_file["dp"].astype(np.float64)
            err = norms.l2(mesh, dp - dref) / norms.l2(mesh, dref)
            row = {"form": name, "amp": amp, "K": mesh.K, "N": N, "steps": STEPS,
                   "p_rel_l2": float(err), "bar": bar, "ok": bool(err <= bar),
                   "t_rel_diff": float(abs(t / float(ref_file["t"]) - 1))}
            rows.append(row)
            print(json.dumps(row), flush=True)
            dg.dg_destroy(ctx)
    return rows


if __name__ == "__main__":
    if len(sys.argv) != 3 or sys.argv[1] not in ("oracle", "gpu"):
        sys.exit("usage: precision_n5_subsample.py oracle|gpu <dir>")
    if sys.argv[1] == "oracle":
        oracle(sys.argv[2])
    else:
        rows = gpu(sys.argv[2])
        sys.exit(0 if all(r["ok"] for r in rows) else 1)
