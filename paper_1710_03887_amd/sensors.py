"""Sensor study of Section 3: the mouthpiece pulse recorded at sensor points
around the trumpet in several outer domains, and the domains compared
through the amplitude spectra of those recordings.

Section 3 places the instrument in full domains (Type A: box, sphere, ...)
and in domains that keep only the region in front of the bell (Type B), runs
the same pulse in each, and compares the pressure spectra at sensors near the
bell and near the outer boundary (Table 2 gives each sensor's distance from
the bell and from the boundary): matching spectra mean the boundary
treatment let the pulse out without disturbing the solution.  Here the
domains are the synthetic trumpet domains of this package (Type A: box,
sphere of radius 1.5, cone, spherical cone; Type B: half box, half cone),
the sensors stand-ins placed by their relation to
the bell plane (x = 1): three at the same place in every domain, and on the
axis a pair 2 cm and 1 cm before each domain's own far wall, and every
signal is recorded every step by the library's probe kernel inside the
captured step graph, with one fixed time step shared by all domains so that
the spectra share their frequency bins.

    python -m paper_1710_03887_amd.sensors [--amps 0.005,0.02] [--t-end 3.0] [--curved]
    python -m paper_1710_03887_amd.sensors --quadrature --N 1 --amps 0.005,0.02,0.1

With --quadrature the runs use the paper's own discretization (weak form with
Gauss quadrature, RK2; DG_SETUP_QUADRATURE), which carries the 10% pulse that
the unlimited nodal scheme does not; the summary then also compares each
amplitude's spectra, rescaled by the amplitude ratio, with the smallest
amplitude's (a linear response gives 0 dB: growth there is the pulse's own
nonlinearity plus whatever the boundary sends back).

With --curved the study compares the spherical domain with flat side faces
against the same mesh with its side faces laid onto the sphere (curved
isoparametric elements), adding a sensor pair 5 cm and 4 cm inside the
curved side wall.

Prints one JSON line per domain run and a summary line: per sensor and
domain the peak |p'| and the spectrum in dB re 20 micropascal (p0 standing
for one atmosphere) at octave-spaced frequencies, and the mean |dB
difference| of each domain from the box over the band where the box's
spectrum lies within 60 dB of its peak.
"""
import argparse
import json
import math
import time

import numpy as np

from . import _lib as dg

GAMMA, RHO0, P0 = 1.4, 1.0, 1.0 / 1.4
ALPHA = 2 * np.pi * 565.0 / 343.0
HZ = 343.0            # one time unit is 1/343 s (lengths in metres, c0 = 1)
P_REF = 2e-5 / 101325.0 * P0
# sensors at the same place in every domain ...
SENSORS = {
    # 1 cm in front of the bell plane and 1 cm below the box's top wall (as
    # Table 2 places it); in the other domains it is farther from their
    # boundaries, so differences there against the box include the box's
    # own behaviour next to its wall
    "sensor 1 (1 cm in front of the bell plane, 1 cm below the box's top wall)": (1.01, 0.99, 0.003),
    "sensor 4 (in front of the bell, 0.57 up)": (1.29, 0.57, 0.003),
    "bore (1 cm inside the mouthpiece)": (0.01, 0.0, 0.003),
}
# ... and, per domain, on the axis 2 cm and 1 cm before its own far wall
FAR = ("sensor 2 (on axis, 2 cm before the far wall)", "sensor 3 (on axis, 1 cm before the far wall)")
DOMAINS = (("box", 50_000), ("sphere", 80_000), ("cone", 80_000), ("scone", 80_000),
           ("half", 30_000), ("half-cone", 40_000))


def _torch():
    import torch
    return torch


def far_wall(m, y=0.0, z=0.003):
    """Largest x where the line (x, y, z) crosses a characteristic-outflow
    face: the domain's outer boundary in front of the bell."""
    from workloads import BC_OUTFLOW_CHAR
    fv = np.array([(0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3)])
    k, f = np.nonzero(m["bc"] == BC_OUTFLOW_CHAR)
    tri = m["xyz"][k[:, None], fv[f]]                       # [nf, 3 vertices, 3]
    a, b, c = tri[:, 0], tri[:, 1], tri[:, 2]
    # barycentric coordinates of (y, z) in the face's yz projection
    d = (b[:, 1] - a[:, 1]) * (c[:, 2] - a[:, 2]) - (c[:, 1] - a[:, 1]) * (b[:, 2] - a[:, 2])
    ok = np.abs(d) > 1e-14
    d = np.where(ok, d, 1.0)
    l1 = ((y - a[:, 1]) * (c[:, 2] - a[:, 2]) - (c[:, 1] - a[:, 1]) * (z - a[:, 2])) / d
    l2 = ((b[:, 1] - a[:, 1]) * (z - a[:, 2]) - (y - a[:, 1]) * (b[:, 2] - a[:, 2])) / d
    hit = ok & (l1 >= 0) & (l2 >= 0) & (l1 + l2 <= 1)
    x = a[:, 0] + l1 * (b[:, 0] - a[:, 0]) + l2 * (c[:, 0] - a[:, 0])
    return float(x[hit].max())


# in the spherical domains, a pair 5 cm and 4 cm inside the sphere's side
# wall, on the ray from its centre (0.5, 0, 0) at 60 degrees to the axis
# (closer points fall outside the flat-faced mesh there: its chords lie up to
# about 3 cm inside the sphere)
SIDE = ("side 2 (5 cm inside the sphere's side wall)", "side 3 (4 cm inside the sphere's side wall)")
SIDE_DIR = np.array([0.5, np.sqrt(3.0) / 2.0, 0.0])


def sensor_points(m, side=False):
    xf = far_wall(m)
    pts = list(SENSORS.values()) + [(xf - 0.02, 0.0, 0.003), (xf - 0.01, 0.0, 0.003)]
    if side:
        c, R = np.array([0.5, 0.0, 0.0]), 1.5
        pts += [tuple(c + (R - d) * SIDE_DIR + np.array([0.0, 0.0, 0.003])) for d in (0.05, 0.04)]
    return pts


def setup(kind, target_K, amp, N=4, side=False, quadrature=False):
    """kind: one of the trumpet_domain kinds, or 'sphere-curved' (the
    spherical domain with its side faces laid onto the sphere as curved
    elements)."""
    from workloads import trumpet_domain
    torch = _torch()
    m = trumpet_domain(kind.replace("-curved", ""), target_K)
    ctx = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], N, gamma=GAMMA, rho0=RHO0, p0=P0,
                           inflow_amp=amp * P0, inflow_alpha=ALPHA, quadrature=quadrature)
    q = torch.zeros((ctx.K, 5, ctx.Np), dtype=torch.float32, device="cuda")
    res = torch.zeros_like(q)
    if kind.endswith("-curved"):
        from workloads.curved import sphere_domain_map, curved_nodes
        mc = sphere_domain_map(m)
        n = dg.dg_set_curved(ctx, curved_nodes(mc, dg.dg_reference_operators(ctx)["rst"]))
        print(f"{kind}: {n} of {ctx.K} elements curved", flush=True)
    dg.dg_autotune(ctx, q, res)
    pts = sensor_points(m, side)
    dg.dg_probe_setup(ctx, pts)
    return ctx, q, res, pts


def record(ctx, q, res, nsteps, dt, n_sensors, chunk=5000, label=""):
    """The sensors' p' after every step: device [nsteps, n_sensors]."""
    torch = _torch()
    series = torch.empty((nsteps, n_sensors), dtype=torch.float32, device="cuda")
    t, done, t0 = 0.0, 0, time.perf_counter()
    while done < nsteps:
        n = min(chunk, nsteps - done)
        t = dg.dg_run_probes(ctx, q, res, n, dt, t, series[done:done + n])
        done += n
        print(f"{label} step {done}/{nsteps} t={t:.3f} ({time.perf_counter() - t0:.0f} s)",
              flush=True)
    return series, t, time.perf_counter() - t0


def spectra(series):
    torch = _torch()
    n = series.shape[0]
    db = torch.empty((series.shape[1], n // 2 + 1), dtype=torch.float32, device="cuda")
    dg.dg_spectrum(series, P_REF, db)
    return db.double().cpu().numpy()


def main():
    ap = argparse.ArgumentParser(description="sensor spectra of the trumpet pulse per domain")
    ap.add_argument("--amps", default="0.005,0.02", help="inflow amplitudes / p0")
    ap.add_argument("--t-end", type=float, default=3.0)
    ap.add_argument("--N", type=int, default=4)
    ap.add_argument("--curved", action="store_true",
                    help="compare the spherical domain with flat and with curved side faces")
    ap.add_argument("--quadrature", action="store_true",
                    help="the paper's discretization (Gauss quadrature, RK2) instead of the nodal one")
    ap.add_argument("--cfl", type=float, default=None,
                    help="CFL of the shared fixed step (default 0.5 nodal, 0.3 quadrature)")
    args = ap.parse_args()
    cfl = args.cfl if args.cfl is not None else (0.3 if args.quadrature else 0.5)
    torch = _torch()
    names = list(SENSORS) + list(FAR) + (list(SIDE) if args.curved else [])
    domains = (("sphere", 80_000), ("sphere-curved", 80_000)) if args.curved else DOMAINS
    ref_kind = domains[0][0]
    summary = {"sensors": SENSORS, "runs": [], "scheme": "quadrature-RK2" if args.quadrature
               else "nodal-LSERK4", "N": args.N}
    all_db = {}
    for amp in [float(a) for a in args.amps.split(",") if a]:
        ctxs = {kind: setup(kind, K, amp, args.N, args.curved, args.quadrature)
                for kind, K in domains}
        dt = 0.9 * min(dg.dg_stable_dt(c, q, cfl) for c, q, _, _ in ctxs.values())
        nsteps = int(math.ceil(args.t_end / dt))
        freqs = np.arange(nsteps // 2 + 1) / (nsteps * dt) * HZ
        octaves = [f for f in (125, 250, 500, 1000, 2000, 4000, 8000) if f < freqs[-1]]
        bins = [int(np.argmin(np.abs(freqs - f))) for f in octaves]
        db, peak = {}, {}
        for kind, (ctx, q, res, pts) in ctxs.items():
            try:
                s, t, secs = record(ctx, q, res, nsteps, dt, len(names), label=f"{kind} {amp}")
            except dg.DGError as err:   # a non-physical state: reported, domain left out
                print(json.dumps({"amp": amp, "domain": kind, "failed": str(err),
                                  "first_bad_step": dg.dg_last_step(ctx)}), flush=True)
                summary.setdefault("failed", []).append({"amp": amp, "domain": kind})
                dg.dg_destroy(ctx)
                continue
            db[kind] = spectra(s)
            peak[kind] = s.abs().max(dim=0).values.double().cpu().numpy()
            row = {"amp": amp, "domain": kind, "K": ctx.K, "steps": nsteps, "dt": dt, "t_end": t,
                   "sensor_xyz": dict(zip(names, [list(p) for p in pts])),
                   "seconds": secs, "ms_per_step": 1e3 * secs / nsteps,
                   "peak_p_prime": dict(zip(names, peak[kind].tolist())),
                   "db_at_hz": {nm: dict(zip(map(str, octaves), db[kind][i, bins].round(2).tolist()))
                                for i, nm in enumerate(names)}}
            print(json.dumps(row), flush=True)
            summary["runs"].append(row)
            dg.dg_destroy(ctx)
            del q, res
            torch.cuda.empty_cache()
        all_db[amp] = db
        if ref_kind not in db:
            continue
        ref = db[ref_kind]
        for kind in db:
            if kind == ref_kind:
                continue
            diffs = {}
            shared = names if args.curved else list(SENSORS)   # the sensors every domain has
            for i, nm in enumerate(shared):
                band = (ref[i] > ref[i].max() - 60) & (freqs > 20) & (freqs < 4000)
                diffs[nm] = float(np.mean(np.abs(db[kind][i, band] - ref[i, band]))) if band.any() else None
            summary.setdefault(f"mean_abs_db_vs_{ref_kind}", {}).setdefault(str(amp), {})[kind] = diffs
        # reflection indicator of the far wall: sensor 3 (1 cm) against sensor 2 (2 cm)
        pairs = [("sensor3_minus_sensor2_db", len(SENSORS))]
        if args.curved:
            pairs.append(("side3_minus_side2_db", len(SENSORS) + len(FAR)))
        for key, i2 in pairs:
            i3 = i2 + 1
            for kind in db:
                band = (db[kind][i2] > db[kind][i2].max() - 60) & (freqs > 300) & (freqs < 4000)
                summary.setdefault(key, {}).setdefault(str(amp), {})[kind] = \
                    float(np.mean(db[kind][i3, band] - db[kind][i2, band])) if band.any() else None
    # amplitude scaling: each amplitude's spectra lowered by 20 log10(amp / the
    # smallest amp) against the smallest amplitude's, over its band
    amps = sorted(all_db)
    if len(amps) > 1:
        a0 = amps[0]
        for amp in amps[1:]:
            shift = 20.0 * np.log10(amp / a0)
            for kind in all_db[amp]:
                if kind not in all_db[a0]:
                    continue
                d0, d1 = all_db[a0][kind], all_db[amp][kind]
                n = min(d0.shape[1], d1.shape[1])
                vals = {}
                for i, nm in enumerate(names):
                    band = (d0[i, :n] > d0[i, :n].max() - 60)
                    band[:2] = False
                    vals[nm] = float(np.mean(np.abs(d1[i, :n][band] - shift - d0[i, :n][band]))) \
                        if band.any() else None
                summary.setdefault("mean_abs_db_vs_smallest_amp_rescaled", {}) \
                    .setdefault(str(amp), {})[kind] = vals
    print(json.dumps({k: v for k, v in summary.items() if k != "runs"}), flush=True)


if __name__ == "__main__":
    main()
