"""Curved (isoparametric) elements, FP64 -- TEST INFRASTRUCTURE ONLY (see
the package docstring).

Section 3 traces the reflections seen in the spherical outer domain back to
its boundary being built from flat faces, and names curved boundary elements
as the remedy (not used there).  This module states the standard
isoparametric treatment of the nodal scheme:

* geometry: the element map x(r, s, t) is the degree-N polynomial through
  given physical positions of the element's nodes; at every node the
  Jacobian matrix has columns Dr x, Ds x, Dt x, J is its determinant and
  the metric terms d(r, s, t)/d(x, y, z) are its inverse;
* faces: at each face node the outward normal is the gradient of the face's
  reference coordinate (face t = -1: -grad t; s = -1: -grad s;
  r + s + t = -1: +grad(r + s + t); r = -1: -grad r); the unit normal is
  that vector over its length, and the length is sJ / J at the node
  (Fscale), sJ the area element of the face in the same reference face
  coordinates as the straight-sided case;
* right-hand side: the volume term in chain-rule form,
      (div F)(node n) = sum_a sum_d (d r_a / d x_d)(n) (D_a F_d)(n),
  which is the straight-sided operator whenever the metric terms are
  constant; the surface term is the straight-sided one with each face
  node's own normal and Fscale (local Lax-Friedrichs, one lambda per face);
* time step: the rule of the straight-sided scheme, with each element's
  vertex (straight-sided) Fscale (the paper gives no rule; a reading).
"""
import numpy as np

from .euler import flux, ghost_state, normal_flux, primitive, sound_speed
from .operators import vandermonde

# outward reference normal of each face as a combination of grad r, grad s, grad t
FACE_GRAD = np.array([[0.0, 0.0, -1.0], [0.0, -1.0, 0.0], [1.0, 1.0, 1.0], [-1.0, 0.0, 0.0]])


class CurvedGeometry:
    """Per-node geometric factors of the mesh with node positions x [K, Np, 3]
    (oracle node order)."""

    def __init__(self, mesh, x):
        ref = mesh.ref
        x = np.asarray(x, dtype=np.float64)
        cols = [np.einsum("ij,kjd->kid", D, x) for D in (ref.Dr, ref.Ds, ref.Dt)]
        Jm = np.stack(cols, axis=3)                          # [K, Np, x_d, r_a]
        self.x = x
        self.J = np.linalg.det(Jm)                           # [K, Np]
        if np.any(self.J <= 0):
            raise ValueError("curved element with a non-positive Jacobian at a node")
        self.drst_dx = np.linalg.inv(Jm)                     # [K, Np, r_a, x_d]
        g = self.drst_dx[:, ref.Fmask]                       # [K, 4, Nfp, a, d]
        nvec = np.einsum("fa,kfiad->kfid", FACE_GRAD, g)
        self.Fscale = np.linalg.norm(nvec, axis=-1)          # [K, 4, Nfp]
        self.normals = nvec / self.Fscale[..., None]         # [K, 4, Nfp, 3]


def rhs(mesh, geo, q, t, phys, sigma=None):
    """dq/dt [K, 5, Np] of the full state q on the curved geometry `geo`."""
    ref = mesh.ref
    g = phys.gamma
    K, Nfp = mesh.K, ref.Nfp
    qn = np.transpose(q, (0, 2, 1))                          # [K, Np, 5]
    F = flux(qn, g)                                          # [3 (d), K, Np, 5]
    DF = np.stack([np.einsum("ij,dkjv->dkiv", D, F) for D in (ref.Dr, ref.Ds, ref.Dt)])
    div = np.einsum("kiad,adkiv->kiv", geo.drst_dx, DF)     # [K, Np, 5]

    qm = qn[:, ref.Fmask, :]                                 # [K, 4, Nfp, 5]
    flat = qn.reshape(K * ref.Np, 5)
    qp = np.empty_like(qm)
    inner = mesh.mapP >= 0
    qp[inner] = flat[mesh.mapP[inner]]
    nrm = geo.normals
    for tag in np.unique(mesh.bc[mesh.EToE < 0]):
        sel = (mesh.EToE < 0) & (mesh.bc == tag)
        qp[sel] = ghost_state(int(tag), qm[sel], nrm[sel], phys, t)
    fm = normal_flux(qm, nrm, g)
    fp = normal_flux(qp, nrm, g)
    unm = np.abs(np.sum(primitive(qm, g)[..., 1:4] * nrm, axis=-1)) + sound_speed(qm, g)
    unp = np.abs(np.sum(primitive(qp, g)[..., 1:4] * nrm, axis=-1)) + sound_speed(qp, g)
    lam = np.maximum(unm, unp).max(axis=2, keepdims=True)    # [K, 4, 1]
    dF = 0.5 * ((fm - fp) - lam[..., None] * (qm - qp)) * geo.Fscale[..., None]
    lifted = ref.LIFT @ dF.reshape(K, 4 * Nfp, 5)
    out = np.transpose(-div + lifted, (0, 2, 1)).copy()
    if sigma is not None:
        out -= sigma[:, None, :] * (q - phys.q0[None, :, None])
    return out


def locate(mesh, geo, points, curved_rows):
    """Element [n] and reference coordinates [n, 3] of each point: the
    element the straight-sided geometry gives (oracle.probes.locate); in an
    element of `curved_rows` (a boolean [K] mask) the reference point solves
    x(r) = point for that element's curved map, by Newton's method from the
    straight-sided estimate with the map's exact derivative."""
    from .probes import locate as locate_straight
    ref = mesh.ref
    elem, rst = locate_straight(mesh, points)
    Vinv = np.linalg.inv(ref.V)
    pts = np.atleast_2d(np.asarray(points, dtype=np.float64))
    for p, k in enumerate(elem):
        if k < 0 or not curved_rows[k]:
            continue
        xe, r = geo.x[k], rst[p].copy()
        for _ in range(50):
            V, Vr, Vs, Vt = vandermonde(ref.N, r[None])
            f = (V @ Vinv @ xe)[0] - pts[p]
            Jm = np.stack([(D @ Vinv @ xe)[0] for D in (Vr, Vs, Vt)], axis=1)
            dr = np.linalg.solve(Jm, f)
            r -= dr
            if np.abs(dr).max() <= 1e-13:
                break
        else:
            raise ValueError(f"point {p}: the curved map of element {k} did not invert")
        rst[p] = r
    return elem, rst
