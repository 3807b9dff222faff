"""Pins of the quadrature-scheme oracle (oracle/quadrature.py).

* the rules integrate every monomial of degree <= 2N (tetrahedron) and
  <= 2N + 1 (face) exactly -- against the exact rational integrals;
* a uniform (free-stream) state has zero right-hand side on a jittered mesh;
* the weak form conserves mass, momentum and energy exactly on a periodic box;
* for a continuous polynomial state of degree <= N with constant velocity the
  flux is itself a polynomial of degree <= N, so the weak form integrated
  exactly equals the nodal strong form (the other oracle route) on every
  element away from the boundary;
* the RK2 step on y' = z y multiplies by 1 + z + z^2/2.
"""
import numpy as np
import pytest

from oracle import euler, norms
from oracle.mesh import Mesh
from oracle.operators import RefElement, tet_monomial_integral, tri_monomial_integral, monomial_exponents
from oracle.quadrature import QuadScheme, tet_rule, tri_rule
from workloads import box_kuhn


@pytest.mark.parametrize("N", [1, 2])
def test_rules_exact(N):
    x, w = tet_rule(N)
    assert abs(w.sum() - 4 / 3) < 1e-14
    for (a, b, c) in monomial_exponents(2 * N):
        got = np.sum(w * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c)
        assert abs(got - float(tet_monomial_integral(a, b, c))) < 1e-13
    lam, wf = tri_rule(N)
    assert abs(wf.sum() - 2) < 1e-14 and np.all(wf > 0) and np.all(lam >= 0)
    u, v = 2 * lam[:, 1] - 1, 2 * lam[:, 2] - 1
    for A in range(2 * N + 2):
        for B in range(2 * N + 2 - A):
            assert abs(np.sum(wf * u ** A * v ** B) - float(tri_monomial_integral(A, B))) < 1e-13
    # and not one degree higher in every direction
    errs = [abs(np.sum(w * x[:, 2] ** (2 * N + 2)) - float(tet_monomial_integral(0, 0, 2 * N + 2)))]
    assert max(errs) > 1e-6


@pytest.mark.parametrize("N", [1, 2])
def test_free_stream(N):
    ref = RefElement(N)
    m = box_kuhn(3, jitter=0.08, seed=1)
    mesh = Mesh(ref, m["xyz"], m["EToV"], m["bc"])
    phys = euler.Physics(u0=(0.2, -0.1, 0.05))
    q = np.broadcast_to(phys.q0[None, :, None], (mesh.K, 5, ref.Np)).copy()
    assert np.abs(QuadScheme(mesh).rhs(q, 0.0, phys)).max() < 1e-12


def test_conservation_periodic():
    ref = RefElement(2)
    m = box_kuhn(3, jitter=0.05, seed=2, periodic=True)
    mesh = Mesh(ref, m["xyz"], m["EToV"], m["bc"])
    phys = euler.Physics()
    from workloads import gaussian_pulse
    prim = gaussian_pulse(mesh.x, 0.1 * phys.p0, 0.4, center=(0.1, -0.2, 0.05))
    prim[..., 1] = 0.2 * np.sin(np.pi * mesh.x[..., 1])
    q = euler.initial_state(prim, phys.gamma)
    rates = norms.totals(mesh, QuadScheme(mesh).rhs(q, 0.0, phys))
    assert np.abs(rates).max() < 1e-12, rates


@pytest.mark.parametrize("N", [1, 2])
def test_equals_nodal_form_for_polynomial_flux(N):
    ref = RefElement(N)
    m = box_kuhn(4, jitter=0.06, seed=3)
    mesh = Mesh(ref, m["xyz"], m["EToV"], m["bc"])
    phys = euler.Physics()
    x, y, z = mesh.x[..., 0], mesh.x[..., 1], mesh.x[..., 2]
    prim = np.zeros(mesh.x.shape[:2] + (5,))
    prim[..., 0] = 1.0 + 0.05 * x - 0.03 * y + (0.02 * x * z if N >= 2 else 0.0)
    prim[..., 1:4] = (0.1, 0.05, -0.02)
    prim[..., 4] = phys.p0 * (1 + 0.04 * z + 0.02 * y + (0.03 * y * y if N >= 2 else 0.0))
    q = euler.initial_state(prim, phys.gamma)
    inner = np.all(mesh.EToE >= 0, axis=1)
    assert inner.sum() > 10
    rq = QuadScheme(mesh).rhs(q, 0.0, phys)[inner]
    rn = euler.rhs(mesh, q, 0.0, phys)[inner]
    assert np.abs(rq - rn).max() < 1e-11 * np.abs(rn).max()


def test_rk2_stability_polynomial():
    class Lin:
        def rhs(self, q, t, phys):
            return -0.7 * q
    s = QuadScheme.__new__(QuadScheme)
    s.rhs = Lin().rhs
    q = np.array([1.0, 2.0])
    z = -0.7 * 0.3
    assert np.allclose(QuadScheme.rk2_step(s, q, 0.0, 0.3, None), (1 + z + z * z / 2) * q, rtol=1e-15)
