"""Inputs of the 100-step accuracy gates: the trumpet in the box reduced to
19,530 tetrahedra, at N = 4 (the throughput workload's order) and N = 5 (the
precision workload's order).  Only meshes, physical parameters and primitive
initial fields are defined here; the expected results are written by
tests/golden/make_gates.py with the FP64 oracle alone, and the GPU tests run
the library from the same inputs.

Cases (Section 2.4 pulse, Appendix A scheme, LSERK4 at CFL 0.5, 100 steps,
each side taking its own time steps):

* c2_inflow   N = 4: fluid at rest, the raised-cosine mouthpiece pulse of
  0.1 p0 from t = 0 (the throughput run's initial condition);
* c2_pulses   N = 4: the same inflow plus Gaussian pressure pulses of 0.1 p0
  in the bell mouth (width 0.1) and next to the box's far face (width 0.15,
  centre 0.15 inside x = 1.8), so that wall, inflow and characteristic
  outflow faces all carry signal within the 100 steps (t_end is about 0.01:
  a wave started at the bell would not reach the outer boundary in time);
* c3_amp*     N = 5: a Gaussian pressure pulse of amplitude A (width 0.2, in
  the bell) with the mouthpiece pulse of the same amplitude, started a
  quarter inflow period in, for A = 0.5 %, 2 % and 10 % of p0;
* c4_*        N = 3: members of the batched ensemble on coarsened domains
  (box, sphere of radius 1.5, half domain; about 1,500 tetrahedra each): the
  quiet fluid with a weak bump near the bore, the mouthpiece pulse at the
  member's amplitude a_i = p0 10^(-3 + 2 i / 15) (i = 0..15: 0.1 % to 10 %),
  started inside the pulse (t = 0.12); the smallest amplitude on the box,
  the median on the sphere, the largest on the half domain.
"""
import numpy as np

TARGET_K = 20_000
STEPS = 100
CFL = 0.5
ALPHA = 2 * np.pi * 565.0 / 343.0          # the pulse's angular frequency (c = 1 units)
QUARTER = 0.25 * 2 * np.pi / ALPHA

# member amplitudes of the batched ensemble (fractions of p0)
ENSEMBLE_AMPS = 10.0 ** (-3.0 + 2.0 * np.arange(16) / 15.0)
ENSEMBLE_T0 = 0.12
ENSEMBLE_BUMP = ((0.02, 0.08, (0.1, 0.0, 0.0)),)
ENSEMBLE_SAMPLES = (("box", 0), ("sphere", 7), ("half", 15))   # (geometry, member)

CASES = {
    "c2_inflow": dict(N=4, amp=0.1, t0=0.0, pulses=()),
    "c2_pulses": dict(N=4, amp=0.1, t0=0.0,
                      pulses=((0.1, 0.1, (1.0, 0.0, 0.0)), (0.1, 0.15, (1.65, 0.55, 0.35)))),
    "c3_amp0.005": dict(N=5, amp=0.005, t0=QUARTER, pulses=((0.005, 0.2, (0.85, 0.05, 0.0)),)),
    "c3_amp0.02": dict(N=5, amp=0.02, t0=QUARTER, pulses=((0.02, 0.2, (0.85, 0.05, 0.0)),)),
    "c3_amp0.1": dict(N=5, amp=0.1, t0=QUARTER, pulses=((0.1, 0.2, (0.85, 0.05, 0.0)),)),
}
for _kind, _i in ENSEMBLE_SAMPLES:
    CASES[f"c4_{_kind}_m{_i}"] = dict(N=3, amp=float(ENSEMBLE_AMPS[_i]), t0=ENSEMBLE_T0,
                                      pulses=ENSEMBLE_BUMP, domain=(_kind, 1500))


def mesh(case=None):
    """The case's mesh (default: the 19,530-tet trumpet in the box)."""
    from workloads import trumpet_domain
    kind, target = CASES[case].get("domain", ("box", TARGET_K)) if case else ("box", TARGET_K)
    return trumpet_domain(kind, target)


def physics(case):
    """Ambient rho0 = 1, p0 = 1/1.4 (c0 = 1); inflow amplitude as a fraction of p0."""
    from oracle import euler
    return euler.Physics(amp=CASES[case]["amp"] / 1.4, alpha=ALPHA)


def initial_primitive(case, x, rho0=1.0, p0=1.0 / 1.4, gamma=1.4):
    """(rho, u, v, w, p) at points x [..., 3]: fluid at rest, the case's
    Gaussian pressure pulses summed, isentropic density."""
    x = np.asarray(x, dtype=np.float64)
    p = np.full(x.shape[:-1], p0)
    for amp, width, centre in CASES[case]["pulses"]:
        p = p + amp * p0 * np.exp(-np.sum((x - np.asarray(centre)) ** 2, axis=-1) / width ** 2)
    out = np.zeros(x.shape[:-1] + (5,))
    out[..., 0] = rho0 * (p / p0) ** (1.0 / gamma)
    out[..., 4] = p
    return out
