"""Pins for the oracle's semi-discrete operator f(q) and its boundary states.

Independent facts used, at every order the hot path runs (N = 2..5):
free-stream preservation, exact conservation on periodic and closed-wall
boxes (round-off scaled by the monomial Vandermonde's conditioning), the
exact translating isentropic vortex (consistency rate in h and geometric
convergence in N of the whole interior operator); and homogeneity of degree
one of the Euler flux, rotation invariance, the algebra of the outflow and wall ghosts,
the linear-acoustic response of a duct to the mouthpiece inflow, and the
values printed in the paper.
"""
import json
import os

import numpy as np
import pytest

from oracle.operators import RefElement
from oracle.mesh import Mesh, MeshError
from oracle import euler, timestep, norms
from workloads import box_kuhn, gaussian_pulse, isentropic_vortex, plane_wave
from workloads import BC_OUTFLOW_CHAR, BC_WALL, BC_PASSTHRU, BC_INFLOW

HERE = os.path.dirname(__file__)
_REFS = {}


def ref_of(N):
    if N not in _REFS:
        _REFS[N] = RefElement(N)
    return _REFS[N]


def make_mesh(N, m):
    return Mesh(ref_of(N), m["xyz"], m["EToV"], m["bc"])


def uniform_state(mesh, phys):
    return np.broadcast_to(phys.q0[None, :, None], (mesh.K, 5, mesh.ref.Np)).copy()


def roundoff(N):
    """FP64 round-off level of the oracle's operators at order N: the
    monomial Vandermonde is inverted explicitly, so errors of a few eps are
    amplified by its condition number (38, 410, 4.8e3, 5.6e4 at N = 2..5);
    a factor 20 above eps * cond(V)."""
    return 20.0 * np.finfo(float).eps * np.linalg.cond(ref_of(N).V)


@pytest.mark.parametrize("N", [2, 3, 4, 5])
@pytest.mark.parametrize("u0", [(0.0, 0.0, 0.0), (0.3, 0.2, 0.1)])
def test_free_stream(N, u0):
    mesh = make_mesh(N, box_kuhn(4, jitter=0.05, seed=1))
    phys = euler.Physics(u0=u0)
    r = euler.rhs(mesh, uniform_state(mesh, phys), 0.0, phys)
    assert np.abs(r).max() < roundoff(N)


def _conservation_rates(mesh, q, phys):
    """Rates of the conserved totals and their round-off scale (the same
    totals of |rhs|)."""
    r = euler.rhs(mesh, q, 0.0, phys)
    return norms.totals(mesh, r), norms.totals(mesh, np.abs(r))


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_conservation_periodic(N):
    mesh = make_mesh(N, box_kuhn(3, jitter=0.05, seed=2, periodic=True))
    phys = euler.Physics()
    prim = gaussian_pulse(mesh.x, 0.1 * phys.p0, 0.4, center=(0.1, -0.2, 0.05))
    prim[..., 1] = 0.2 * np.sin(np.pi * mesh.x[..., 1])
    q = euler.initial_state(prim, phys.gamma)
    rates, scale = _conservation_rates(mesh, q, phys)
    assert (np.abs(rates) < roundoff(N) * scale).all(), rates / scale


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_conservation_walls(N):
    """Closed slip-wall box: mass and energy are conserved (the mirror
    ghost carries no mass or energy flux); momentum is not (wall pressure)."""
    mesh = make_mesh(N, box_kuhn(3, jitter=0.05, seed=3, bc=BC_WALL))
    phys = euler.Physics()
    prim = gaussian_pulse(mesh.x, 0.1 * phys.p0, 0.4, center=(0.1, -0.2, 0.05))
    prim[..., 1:4] = 0.1 * np.cos(mesh.x)
    q = euler.initial_state(prim, phys.gamma)
    rates, scale = _conservation_rates(mesh, q, phys)
    assert (np.abs(rates[[0, 4]]) < roundoff(N) * scale[[0, 4]]).all(), rates / scale
    assert (np.abs(rates[1:4]) > 1e-6 * scale[1:4]).any()


def test_homogeneity():
    mesh = make_mesh(2, box_kuhn(3, jitter=0.05))
    s = 1.4
    p1 = euler.Physics()
    p2 = euler.Physics(rho0=s * p1.rho0, p0=s * p1.p0)
    prim = gaussian_pulse(mesh.x, 0.1 * p1.p0, 0.3)
    prim[..., 1] = 0.05
    q = euler.initial_state(prim, p1.gamma)
    r1 = euler.rhs(mesh, q, 0.0, p1)
    r2 = euler.rhs(mesh, s * q, 0.0, p2)
    assert np.allclose(r2, s * r1, rtol=0, atol=1e-13 * np.abs(r1).max())


def _rotation(a, b, c):
    def R(axis, th):
        m = np.eye(3)
        i, j = [k for k in range(3) if k != axis]
        m[i, i] = m[j, j] = np.cos(th)
        m[i, j], m[j, i] = -np.sin(th), np.sin(th)
        return m
    return R(0, a) @ R(1, b) @ R(2, c)


def test_rotation_invariance():
    m = box_kuhn(3, jitter=0.05, seed=4)
    Rm = _rotation(0.3, -0.7, 1.1)
    m2 = dict(m, xyz=m["xyz"] @ Rm.T + np.array([0.3, -0.1, 2.0]))
    mesh1, mesh2 = make_mesh(2, m), make_mesh(2, m2)
    phys = euler.Physics()
    prim1 = gaussian_pulse(mesh1.x, 0.1 * phys.p0, 0.3, center=(0.2, 0.1, -0.1))
    prim1[..., 1:4] = 0.1 * np.sin(mesh1.x[..., ::-1])
    prim2 = prim1.copy()
    prim2[..., 1:4] = prim1[..., 1:4] @ Rm.T
    r1 = euler.rhs(mesh1, euler.initial_state(prim1, phys.gamma), 0.0, phys)
    r2 = euler.rhs(mesh2, euler.initial_state(prim2, phys.gamma), 0.0, phys)
    r1_rot = r1.copy()
    r1_rot[:, 1:4] = np.einsum("ij,kjn->kin", Rm, r1[:, 1:4])
    assert np.allclose(r2, r1_rot, atol=1e-12 * np.abs(r1).max())


def test_vertex_relabelling_and_orientation():
    """Relabel every element's vertices cyclically (flipping half of them):
    the operator is the same at the same physical nodes."""
    m = box_kuhn(3, jitter=0.05, seed=5)
    perm = [1, 2, 3, 0]
    # face f of the new labelling = old face with vertex set perm[face]
    fv = ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))
    old_of = [fv.index(tuple(sorted(perm[v] for v in f))) for f in fv]
    m2 = {"xyz": m["xyz"][:, perm], "EToV": m["EToV"][:, perm], "bc": m["bc"][:, old_of]}
    mesh1, mesh2 = make_mesh(2, m), make_mesh(2, m2)
    phys = euler.Physics()
    q1 = euler.initial_state(gaussian_pulse(mesh1.x, 0.1 * phys.p0, 0.3), phys.gamma)
    q2 = euler.initial_state(gaussian_pulse(mesh2.x, 0.1 * phys.p0, 0.3), phys.gamma)
    r1 = euler.rhs(mesh1, q1, 0.0, phys)
    r2 = euler.rhs(mesh2, q2, 0.0, phys)
    for k in range(mesh1.K):
        d = np.linalg.norm(mesh1.x[k][:, None] - mesh2.x[k][None], axis=-1)
        j = d.argmin(axis=1)
        assert d.min(axis=1).max() < 1e-12
        assert np.allclose(r1[k], r2[k][:, j], atol=1e-11)


def test_mesh_errors():
    m = box_kuhn(2)
    bad = dict(m, bc=m["bc"].copy())
    bad["bc"][bad["bc"] > 0] = 0
    with pytest.raises(MeshError):
        make_mesh(2, bad)
    flat = dict(m, xyz=m["xyz"].copy())
    flat["xyz"][0, 3] = flat["xyz"][0, 0]
    with pytest.raises(MeshError):
        make_mesh(2, flat)


def _vortex_residual(N, n):
    Lz = 10.0 * 3 / n
    m = box_kuhn((n, n, 3), lo=(-5, -5, 0), hi=(5, 5, Lz), periodic=True)
    mesh = make_mesh(N, m)
    phys = euler.Physics(rho0=1.0, p0=1.0)
    # centre off the mesh planes, so that no node sits where the periodic
    # image switches (the field is ~1e-5 there, not exactly periodic)
    kw = dict(beta=5.0, center=(0.31, 0.17), velocity=(1.0, 0.5), period=(10.0, 10.0))
    q = euler.initial_state(isentropic_vortex(mesh.x, 0.0, **kw), phys.gamma)
    eps = 1e-5
    qa = euler.initial_state(isentropic_vortex(mesh.x, eps, **kw), phys.gamma)
    qb = euler.initial_state(isentropic_vortex(mesh.x, -eps, **kw), phys.gamma)
    dqdt = (qa - qb) / (2 * eps)
    e = euler.rhs(mesh, q, 0.0, phys) - dqdt
    return np.sqrt(sum(norms.l2(mesh, e[:, v]) ** 2 for v in range(5)))


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_vortex_consistency_rate(N):
    """The residual f(q_exact) - dq_exact/dt of the nodal strong form is the
    derivative of an interpolation error, O(h^N): halving h (8 -> 16 hexes
    across the 10 x 10 period) gains at least N - 1/2 (observed 2.0, 3.2,
    3.8, 5.2 at N = 2..5)."""
    e1, e2 = _vortex_residual(N, 8), _vortex_residual(N, 16)
    rate = np.log2(e1 / e2)
    assert rate > N - 0.5, (e1, e2, rate)


def test_vortex_p_convergence():
    """On a fixed mesh (12 x 12 hexes across the period) the same residual
    falls at least geometrically with the order: each order at least halves
    it (observed ratios 0.33, 0.28, 0.33 from N = 2 to 5), so it decreases
    monotonically -- spectral convergence of the smooth solution."""
    e = [_vortex_residual(N, 12) for N in (2, 3, 4, 5)]
    ratios = [e[i + 1] / e[i] for i in range(3)]
    assert all(r < 0.5 for r in ratios), (e, ratios)


def test_outflow_ghost_algebra():
    """Outgoing plane acoustic state: the ghost equals it (no reflection);
    incoming one: the ghost is the ambient state; the wall ghost mirrors."""
    phys = euler.Physics()
    rng = np.random.default_rng(0)
    n = rng.standard_normal((20, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    A = 1e-3
    Z0, c0 = phys.rho0 * phys.c0, phys.c0
    for sign, expect_self in ((1, True), (-1, False)):
        prim = np.zeros((20, 5))
        prim[:, 0] = phys.rho0 + A / c0 ** 2
        prim[:, 1:4] = sign * (A / Z0) * n
        prim[:, 4] = phys.p0 + A
        qm = euler.conserved(prim, phys.gamma)
        g = euler.ghost_state(euler.OUTFLOW_CHAR, qm, n, phys, 0.0)
        target = qm if expect_self else np.broadcast_to(phys.q0, qm.shape)
        assert np.allclose(g, target, atol=1e-14)
    qm = euler.conserved(np.c_[1.1 * np.ones(20), rng.standard_normal((20, 3)) * 0.1,
                               0.8 * np.ones(20)], phys.gamma)
    g = euler.ghost_state(euler.WALL, qm, n, phys, 0.0)
    assert np.allclose(g[:, 0], qm[:, 0]) and np.allclose(g[:, 4], qm[:, 4])
    un_m = np.sum(qm[:, 1:4] * n, 1)
    un_g = np.sum(g[:, 1:4] * n, 1)
    assert np.allclose(un_g, -un_m, atol=1e-15)
    assert np.allclose(g[:, 1:4] - un_g[:, None] * n, qm[:, 1:4] - un_m[:, None] * n)


def _run_to(mesh, q, phys, T, cfl=0.5):
    """Fixed-step run to time T with the CFL-rule step of the start state."""
    n = int(np.ceil(T / timestep.stable_dt(mesh, q, phys, cfl)))
    q, t, _ = timestep.run(mesh, q, phys, n, dts=[T / n] * n)
    return q


def _duct(N, nx, L, bc_left, bc_right):
    """A one-hex-wide duct along x; slip walls on the four sides keep a
    plane wave along x an exact solution."""
    h = L / nx
    bc = {"x-": bc_left, "x+": bc_right, "y-": BC_WALL, "y+": BC_WALL,
          "z-": BC_WALL, "z+": BC_WALL}
    return make_mesh(N, box_kuhn((nx, 1, 1), lo=(0, 0, 0), hi=(L, h, h), bc=bc))


@pytest.mark.parametrize("bc_right,expect_reflection", [(BC_OUTFLOW_CHAR, False),
                                                       (BC_PASSTHRU, False),
                                                       (BC_WALL, True)])
def test_normal_incidence_reflection(bc_right, expect_reflection):
    """A small right-going plane pulse leaves through an outflow or
    pass-through face with almost no reflection; a wall sends it back with
    R = +1 (pressure doubling at the wall)."""
    mesh = _duct(2, 16, 1.5, BC_WALL, bc_right)
    phys = euler.Physics()
    A = 1e-5 * phys.p0
    xs = mesh.x[..., 0]
    pp = A * np.exp(-((xs - 0.75) / 0.15) ** 2)
    prim = np.zeros(mesh.x.shape[:2] + (5,))
    prim[..., 0] = phys.rho0 + pp / phys.c0 ** 2
    prim[..., 1] = pp / (phys.rho0 * phys.c0)
    prim[..., 4] = phys.p0 + pp
    q = euler.initial_state(prim, phys.gamma)
    q = _run_to(mesh, q, phys, 1.3)
    pres = norms.pressure(q, phys.gamma) - phys.p0
    peak = np.abs(pres).max() / A
    if expect_reflection:
        # the pulse has come back: centred at 1.5 - (0.75 + 1.3 - 1.5) = 0.95
        k = np.argmax(np.abs(pres).max(axis=1))
        assert peak > 0.85 and abs(mesh.x[k, :, 0].mean() - 0.95) < 0.15
        assert pres.flat[np.abs(pres).argmax()] > 0
    else:
        assert peak < 5e-3, peak


def test_inflow_duct_linear_response():
    """Mouthpiece inflow (Eqs. 5-7) into a duct: in the linear limit the
    interior pressure is the pulse delayed by x/c0."""
    alpha = 2 * np.pi
    phys = euler.Physics(amp=1e-5 / 1.4, alpha=alpha)
    mesh = _duct(3, 16, 1.5, BC_INFLOW, BC_OUTFLOW_CHAR)
    q = uniform_state(mesh, phys)
    T = 1.2
    q = _run_to(mesh, q, phys, T)
    pres = norms.pressure(q, phys.gamma) - phys.p0
    xs = mesh.x[..., 0]
    tau = T - xs / phys.c0
    expect = np.where((tau >= 0) & (tau < 2 * np.pi / alpha),
                      phys.amp * 0.5 * (1 - np.cos(alpha * tau)), 0.0)
    err = np.abs(pres - expect).max() / phys.amp
    assert err < 0.03, err


def test_printed_values():
    g = json.load(open(os.path.join(HERE, "golden", "paper_printed_values.json")))
    ic = g["initial_state"]
    q = euler.conserved(np.array([ic["rho0"], 0, 0, 0, ic["p0"]]), ic["gamma"])
    assert abs(q[4] - ic["E0"]) < 1e-15
    # the scaling: c0 = sqrt(gamma p0 / rho0) = 1
    assert abs(np.sqrt(ic["gamma"] * ic["p0"] / ic["rho0"]) - 1.0) < 1e-15
    pu = g["pulse"]
    phys = euler.Physics(rho0=1.4, p0=1.0, amp=pu["peak_over_p0"], alpha=1.0)
    peak = euler.inflow_pressure(phys, np.pi) - 1.0
    assert abs(peak * pu["atmosphere_Pa"] - 10132.5) < 1e-9
    assert abs(peak * pu["atmosphere_Pa"] - pu["peak_Pa_approx"]) / 1e4 < 0.02
    for pa, pct in g["amplitudes_in_percent_of_p0"].items():
        if pa.startswith("_"):
            continue
        assert abs(100 * float(pa) / pu["atmosphere_Pa"] - pct) < 5e-4 * pct


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_dt_rule_is_stable_with_margin(N):
    """The time-step rule is a choice (the paper gives none), but two facts
    bound it.  Linearized about the ambient state (central differences; the
    Lax-Friedrichs speed's kink at u = 0 multiplies a jump that vanishes
    there), the semi-discrete operator J of the box with characteristic
    faces has its spectrum in the closed left half plane, the energy
    stability of the upwind-type flux; and dt at CFL 0.5 puts every dt
    lambda inside the stability region |R(z)| <= 1 of the five-stage scheme
    (R from its coefficients, Appendix A, Eq. 12).  The largest stable CFL
    lies between 1 and 4 at every order (observed 1.81, 2.10, 2.29, 2.44 at
    N = 2..5): the (N+1)^2 Fscale (|u| + c) scaling tracks the spectral
    radius, so the margin does not shrink with N (with (N+1) instead, CFL
    0.5 is unstable at N = 4)."""
    mesh = make_mesh(N, box_kuhn(1, jitter=0.05, seed=1))
    phys = euler.Physics()
    q0 = uniform_state(mesh, phys)
    n, eps = q0.size, 1e-6
    J = np.empty((n, n))
    for j in range(n):
        d = np.zeros(n)
        d[j] = eps
        d = d.reshape(q0.shape)
        J[:, j] = ((euler.rhs(mesh, q0 + d, 0.0, phys) - euler.rhs(mesh, q0 - d, 0.0, phys))
                   / (2 * eps)).ravel()
    lam = np.linalg.eigvals(J)
    assert lam.real.max() <= 1e-9 * np.abs(lam).max()

    def amp(cfl):
        z = cfl * timestep.stable_dt(mesh, q0, phys, 1.0) * lam
        y, res = np.ones_like(z), np.zeros_like(z)
        for a, b in zip(timestep.A, timestep.B):   # the scheme on y' = lambda y
            res = a * res + z * y
            y = y + b * res
        return np.abs(y).max()

    assert amp(0.5) <= 1 + 1e-9
    assert amp(1.0) <= 1 + 1e-9 and amp(4.0) > 1 + 1e-9
