"""Time integration of dc/dt = f(c) (Appendix A, Eq. 12) -- oracle.

The paper advances its ODE system with a second-order Runge-Kutta scheme
(Section 1.1); the hot path uses the five-stage, fourth-order, 2N-storage
Runge-Kutta scheme of Carpenter & Kennedy (1994).  For i = 1..5:

    res <- a_i res + dt f(q, t + c_i dt);   q <- q + b_i res,

with a_1 = 0, so no residual has to be carried across steps.

Time step (the paper gives none; a choice):
    dt = CFL / max over elements k, faces f, face nodes i of
         (N+1)^2/2 * Fscale_{k,f} * (|u| + c)  evaluated on interior traces.
Pinned by what stability fixes: at CFL 0.5, dt times every eigenvalue of
the linearized operator lies inside the scheme's stability region, and the
largest stable CFL stays between 1 and 4 at N = 2..5.
"""
from fractions import Fraction

import numpy as np

from .euler import primitive, sound_speed

RK4A = (Fraction(0), Fraction(-567301805773, 1357537059087),
        Fraction(-2404267990393, 2016746695238), Fraction(-3550918686646, 2091501179385),
        Fraction(-1275806237668, 842570457699))
RK4B = (Fraction(1432997174477, 9575080441755), Fraction(5161836677717, 13612068292357),
        Fraction(1720146321549, 2090206949498), Fraction(3134564353537, 4481467310338),
        Fraction(2277821191437, 14882151754819))
RK4C = (Fraction(0), Fraction(1432997174477, 9575080441755),
        Fraction(2526269341429, 6820363962896), Fraction(2006345519317, 3224310063776),
        Fraction(2802321613138, 2924317926251))

A = tuple(float(x) for x in RK4A)
B = tuple(float(x) for x in RK4B)
C = tuple(float(x) for x in RK4C)


def lserk_step(f, q, t, dt, res=None):
    """One 5-stage step of y' = f(y, t).  Returns (q_new, res)."""
    q = np.array(q, dtype=np.float64, copy=True)
    res = np.zeros_like(q) if res is None else np.array(res, copy=True)
    for i in range(5):
        res = A[i] * res + dt * f(q, t + C[i] * dt)
        q = q + B[i] * res
    return q, res


def stable_dt(mesh, q, phys, cfl):
    """dt from the interior face traces of q [K, 5, Np]."""
    ref = mesh.ref
    qn = np.transpose(q, (0, 2, 1))[:, ref.Fmask, :]          # [K, 4, Nfp, 5]
    w = primitive(qn, phys.gamma)
    speed = np.linalg.norm(w[..., 1:4], axis=-1) + sound_speed(qn, phys.gamma)
    rate = 0.5 * (ref.N + 1) ** 2 * mesh.Fscale[:, :, None] * speed
    return cfl / rate.max()


def run(mesh, q, phys, nsteps, cfl=None, dts=None, t0=0.0, rhs_fn=None, learned=None,
        sigma=None):
    """Advance nsteps.  dt per step from `dts` if given, else from the CFL
    rule at the start of the step.  Returns (q, t, list of dt)."""
    from .euler import rhs as euler_rhs
    if rhs_fn is None:
        def rhs_fn(qq, tt):
            return euler_rhs(mesh, qq, tt, phys, learned, sigma=sigma)
    t = t0
    used = []
    res = None
    for n in range(nsteps):
        dt = dts[n] if dts is not None else stable_dt(mesh, q, phys, cfl)
        q, res = lserk_step(rhs_fn, q, t, dt, res)
        t = t + dt
        used.append(dt)
    return q, t, used
