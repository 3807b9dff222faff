"""Pins of the oracle's absorbing-layer term (rhs - sigma (q - q0)).

* a uniform state q0 + delta on a periodic box has no flux divergence and no
  face jumps, so its right-hand side is exactly -sigma delta, node by node;
* with a constant rate, n LSERK4 steps multiply delta by R(-sigma dt)^n,
  R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 + z^5/200 the scheme's stability
  polynomial (a closed form, independent of the oracle's stage loop);
* the term vanishes where sigma is zero (the rest of the mesh sees the plain
  operator bit for bit).
"""
import numpy as np

from oracle import euler, timestep
from oracle.mesh import Mesh
from oracle.operators import RefElement
from workloads import box_kuhn, gaussian_pulse


def _uniform(mesh, phys, delta):
    q = np.broadcast_to(phys.q0[None, :, None], (mesh.K, 5, mesh.ref.Np)).copy()
    return q + delta[None, :, None]


def test_uniform_state_relaxes_at_sigma():
    ref = RefElement(3)
    mesh = Mesh(ref, *[box_kuhn(3, jitter=0.05, seed=5, periodic=True)[k] for k in ("xyz", "EToV", "bc")])
    phys = euler.Physics(u0=(0.2, -0.1, 0.05))
    delta = np.array([1e-3, 2e-3, -1e-3, 5e-4, 3e-3])
    sigma = np.random.default_rng(0).uniform(0, 5, size=(mesh.K, ref.Np))
    r = euler.rhs(mesh, _uniform(mesh, phys, delta), 0.0, phys, sigma=sigma)
    assert np.allclose(r, -sigma[:, None, :] * delta[None, :, None], rtol=1e-9, atol=1e-13)


def test_lserk4_decay_matches_stability_polynomial():
    ref = RefElement(2)
    mesh = Mesh(ref, *[box_kuhn(3, jitter=0.0, periodic=True)[k] for k in ("xyz", "EToV", "bc")])
    phys = euler.Physics()
    delta = np.array([1e-3, 0.0, 0.0, 0.0, 2e-3])
    s, dt, n = 3.0, 0.05, 7
    q, _, _ = timestep.run(mesh, _uniform(mesh, phys, delta), phys, n, dts=[dt] * n,
                           sigma=np.full((mesh.K, ref.Np), s))
    z = -s * dt
    R = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24 + z ** 5 / 200
    got = q - phys.q0[None, :, None]
    # the uniform state's flux divergence is zero up to rounding (~1e-14 of p0)
    assert np.abs(got - R ** n * delta[None, :, None]).max() < 1e-13


def test_zero_rate_is_the_plain_operator():
    ref = RefElement(2)
    mesh = Mesh(ref, *[box_kuhn(2, jitter=0.05, seed=3)[k] for k in ("xyz", "EToV", "bc")])
    phys = euler.Physics()
    q = euler.initial_state(gaussian_pulse(mesh.x, 0.1 * phys.p0, 0.4), phys.gamma)
    sigma = np.zeros((mesh.K, ref.Np))
    sigma[:3] = 2.0
    r0 = euler.rhs(mesh, q, 0.0, phys)
    r1 = euler.rhs(mesh, q, 0.0, phys, sigma=sigma)
    assert np.array_equal(r0[3:], r1[3:])
    assert np.allclose(r1[:3], r0[:3] - 2.0 * (q[:3] - phys.q0[None, :, None]), rtol=1e-12)
