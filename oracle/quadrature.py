"""The paper's discretization, FP64 -- TEST INFRASTRUCTURE ONLY (see the
package docstring).

Appendix A states the Galerkin problem on each element in weak form,
    int_K v dq/dt dx = int_K grad(v) . F(q) dx - oint_dK v F* . n ds,
and integrates it with Gauss quadrature: rules exact to degree 2p inside the
element and 2p + 1 on its faces; time is advanced by a second-order
Runge-Kutta scheme.  This module restates that, on the same polynomial space
as the nodal oracle (the order-N nodal basis, built from monomials), plainly:

* rules: inside, the collapsed-coordinate product of Gauss-Jacobi rules
  (scipy's roots) with N + 1 points per direction,
  r = (1+a)(1-b)(1-c)/4 - 1, s = (1+b)(1-c)/2 - 1, t = c with weights
  w_a w_b w_c / 8 (Jacobi weights 1, (1-b), (1-c)^2); on faces Radon's
  symmetric seven-point rule of degree 5 (Radon 1948), whose point set does
  not depend on the order of the face's vertices, so the two elements of a
  face integrate the same numerical flux at the same points (conservation);
* volume term: the nodal polynomial and its flux at the volume points, the
  gradients of the basis functions by the monomial derivative Vandermonde;
* face term: both sides' polynomials at the face's points (the neighbour's
  found by placing the point with its own vertex coordinates and inverting
  its affine map, no orientation tables), the
  ghost state of the face's tag on boundary faces, and the local
  Lax-Friedrichs flux F* . n = (F- . n + F+ . n)/2 + lambda (q- - q+)/2 with
  one lambda per face (largest |u.n| + c over its points and both sides);
* dq/dt = M^-1 [ volume - sum_f Fscale_f face_f ] per element (M the exact
  reference mass matrix; the element's Jacobian cancels);
* time: the two-stage strong-stability-preserving RK2 (Heun) step
  q1 = q + dt L(q, t),  q_new = (q + q1 + dt L(q1, t + dt)) / 2 -- the paper
  names only "RK2"; this variant is the reading.
"""
import numpy as np
from scipy.special import roots_jacobi

from .euler import flux, normal_flux, primitive, sound_speed, ghost_state
from .mesh import FACE_VERTS
from .operators import vandermonde


def tet_rule(N):
    """Points [Nq, 3] and weights [Nq] on the reference tetrahedron."""
    n = N + 1
    a, wa = roots_jacobi(n, 0.0, 0.0)
    b, wb = roots_jacobi(n, 1.0, 0.0)
    c, wc = roots_jacobi(n, 2.0, 0.0)
    A, B, C = np.meshgrid(a, b, c, indexing="ij")
    W = (wa[:, None, None] * wb[None, :, None] * wc[None, None, :]) / 8.0
    r = (1 + A) * (1 - B) * (1 - C) / 4 - 1
    s = (1 + B) * (1 - C) / 2 - 1
    return np.stack([r.ravel(), s.ravel(), C.ravel()], axis=1), W.ravel()


def tri_rule(N):
    """Barycentric coordinates [7, 3] on a face's three vertices and weights
    [7] (face coordinates of area 2): Radon's seven-point rule, exact to
    degree 5 >= 2N + 1 for N <= 2 and symmetric under every permutation of
    the vertices, so both elements sharing a face use the same points."""
    if N > 2:
        raise ValueError("the face rule covers N <= 2")
    r15 = np.sqrt(15.0)
    pts, wts = [(1 / 3, 1 / 3, 1 / 3)], [9 / 40]
    for a, w in (((6 - r15) / 21, (155 - r15) / 1200), ((6 + r15) / 21, (155 + r15) / 1200)):
        b = 1 - 2 * a
        pts += [(b, a, a), (a, b, a), (a, a, b)]
        wts += [w] * 3
    return np.array(pts), 2.0 * np.array(wts)


def _basis(ref, rst):
    """Nodal basis values [n, Np] and reference gradients [3, n, Np] at rst."""
    V = vandermonde(ref.N, ref.rst)[0]
    Vx, Vr, Vs, Vt = vandermonde(ref.N, np.atleast_2d(rst))
    Vinv = np.linalg.inv(V)
    return Vx @ Vinv, np.stack([Vr @ Vinv, Vs @ Vinv, Vt @ Vinv])


class QuadScheme:
    """Precomputed rules and basis values for a mesh."""

    def __init__(self, mesh):
        self.mesh = mesh
        ref = mesh.ref
        self.xq, self.wq = tet_rule(ref.N)
        self.Bv, self.dB = _basis(ref, self.xq)            # [Nq, Np], [3, Nq, Np]
        self.lam, self.wf = tri_rule(ref.N)
        K, Nfq = mesh.K, len(self.wf)
        # face points: reference coordinates in the element and physical points
        self.Bf = np.empty((4, Nfq, ref.Np))
        self.xphys = np.empty((K, 4, Nfq, 3))
        for f, vs in enumerate(FACE_VERTS):
            bary = np.zeros((Nfq, 4))
            bary[:, list(vs)] = self.lam
            self.Bf[f] = _basis(ref, 2.0 * bary[:, 1:] - 1.0)[0]
            self.xphys[:, f] = np.einsum("qv,kvd->kqd", bary, mesh.xyz)
        # neighbour's basis at my face points: the same barycentric weights on
        # the same topological vertices, placed with the neighbour's own vertex
        # coordinates (periodic images included), then its affine map inverted
        self.Bnb = np.zeros((K, 4, Nfq, ref.Np))
        for k in range(K):
            for f, vs in enumerate(FACE_VERTS):
                k2 = mesh.EToE[k, f]
                if k2 < 0:
                    continue
                idx = [int(np.nonzero(mesh.EToV[k2] == mesh.EToV[k, v])[0][0]) for v in vs]
                x = self.lam @ mesh.xyz[k2, idx]                     # [Nfq, 3]
                # x - v0 = J (1 + r) with J = dx/dr: (1 + r) = drst_dx (x - v0)
                rst = (mesh.drst_dx[k2] @ (x - mesh.xyz[k2, 0]).T).T - 1.0
                self.Bnb[k, f] = _basis(ref, rst)[0]

    def rhs(self, q, t, phys):
        """dq/dt [K, 5, Np] of the full state q [K, 5, Np]."""
        mesh, ref = self.mesh, self.mesh.ref
        g = phys.gamma
        qn = np.transpose(q, (0, 2, 1))                       # [K, Np, 5]
        # volume: sum_q w_q sum_a dl_i/dr_a Fc_a
        uq = np.einsum("qi,kiv->kqv", self.Bv, qn)            # [K, Nq, 5]
        F = flux(uq, g)                                       # [3, K, Nq, 5]
        Fc = np.einsum("kad,dkqv->akqv", mesh.drst_dx, F)     # [3, K, Nq, 5]
        vol = np.einsum("aqi,q,akqv->kiv", self.dB, self.wq, Fc)
        # faces
        surf = np.zeros_like(vol)
        for f in range(4):
            qm = np.einsum("qi,kiv->kqv", self.Bf[f], qn)     # [K, Nfq, 5]
            k2 = mesh.EToE[:, f]
            qp = np.einsum("kqi,kiv->kqv", self.Bnb[:, f], qn[np.maximum(k2, 0)])
            n = np.broadcast_to(mesh.normals[:, f, None, :], qm.shape[:2] + (3,))
            for tag in np.unique(mesh.bc[:, f][k2 < 0]):
                sel = (k2 < 0) & (mesh.bc[:, f] == tag)
                qp[sel] = ghost_state(int(tag), qm[sel], n[sel], phys, t)
            fm = normal_flux(qm, n, g)
            fp = normal_flux(qp, n, g)
            sm = np.abs(np.sum(primitive(qm, g)[..., 1:4] * n, axis=-1)) + sound_speed(qm, g)
            sp = np.abs(np.sum(primitive(qp, g)[..., 1:4] * n, axis=-1)) + sound_speed(qp, g)
            lam = np.maximum(sm, sp).max(axis=1)                # [K]
            Fs = 0.5 * (fm + fp) + 0.5 * lam[:, None, None] * (qm - qp)
            surf += mesh.Fscale[:, f, None, None] * np.einsum("qi,q,kqv->kiv", self.Bf[f], self.wf, Fs)
        out = np.einsum("ij,kjv->kiv", ref.Minv, vol - surf)
        return np.transpose(out, (0, 2, 1)).copy()

    def rk2_step(self, q, t, dt, phys):
        q1 = q + dt * self.rhs(q, t, phys)
        return 0.5 * (q + q1 + dt * self.rhs(q1, t + dt, phys))

    def run(self, q, phys, nsteps, cfl=None, dts=None, t0=0.0):
        """nsteps RK2 steps; dt from `dts` or the CFL rule of timestep.stable_dt.
        Returns (q, t, list of dt)."""
        from .timestep import stable_dt
        t, used = t0, []
        for j in range(nsteps):
            dt = dts[j] if dts is not None else stable_dt(self.mesh, q, phys, cfl)
            q = self.rk2_step(q, t, dt, phys)
            t += dt
            used.append(dt)
        return q, t, used
