"""Curved-boundary inputs: meshes whose vertex pre-images are known and a
smooth map of space that places element nodes on a curved boundary.

Geometry only (nothing here evaluates the discretization).  A mesh dict
carries, besides ``xyz``/``EToV``/``bc``:

``param``  float64 [K, 4, 3]  pre-image of each element's vertices
``phi``    callable           the map, points [..., 3] -> points [..., 3]

with ``xyz == phi(param)``.  The curved position of an element node is
``phi`` of the node's pre-image, the affine image of its reference
coordinates in the element's pre-image vertices (``curved_nodes``).  Since
``phi`` is one function of space and the pre-image mesh is conforming, the
nodes that two elements share on a face land on the same points.

``capped_box``: the Kuhn-split box [-1, 1]^3 whose x = 1 face is bent onto
a spherical cap (``cap_map``); elements with x <= x0 stay straight.

``sphere_domain_map``: for the trumpet's spherical domain, whose outer
vertices lie on a sphere and whose side faces are flat chords between
them; see its docstring.
"""
import numpy as np

from .meshes import BC_OUTFLOW_CHAR, box_kuhn


def _smoothstep(u):
    u = np.clip(u, 0.0, 1.0)
    return u * u * (3 - 2 * u)


def cap_map(R=3.0, x0=0.0):
    """Map of the box [-1, 1]^3 that bends its x = 1 face onto the sphere
    of radius R about c = (1 - R, 0, 0) (through (1, 0, 0)):
    x -> x + w(x) (c_x + sqrt(R^2 - y^2 - z^2) - 1), y and z unchanged,
    w = smoothstep((x - x0)/(1 - x0)).  The identity for x <= x0; the side
    faces stay planar."""
    cx = 1.0 - R

    def phi(p):
        p = np.array(p, dtype=np.float64)
        y, z = p[..., 1], p[..., 2]
        w = _smoothstep((p[..., 0] - x0) / (1.0 - x0))
        p[..., 0] += w * (cx + np.sqrt(R * R - y * y - z * z) - 1.0)
        return p
    return phi


def capped_box(n, R=3.0, x0=0.0, bc=BC_OUTFLOW_CHAR):
    """Kuhn-split box [-1, 1]^3 (n^3 hexes, 6 tets each) with its x = 1 face
    bent onto a spherical cap (``cap_map``); ``bc`` as for box_kuhn."""
    m = box_kuhn(n, bc=bc)
    phi = cap_map(R, x0)
    m["param"] = m["xyz"].copy()
    m["xyz"] = np.ascontiguousarray(phi(m["param"]))
    m["phi"] = phi
    m["sphere"] = (np.array([1.0 - R, 0.0, 0.0]), R)
    return m


def curved_nodes(m, rst):
    """Curved node positions [K, Np, 3] for reference nodes rst [Np, 3].

    Elements are taken in the orientation that mesh consumers give them
    (local vertices 1 and 2 swapped where the vertex Jacobian is negative);
    reference vertex order v0 = (-1,-1,-1), v1 = (1,-1,-1), v2 = (-1,1,-1),
    v3 = (-1,-1,1).
    """
    xyz, P = m["xyz"], m["param"].copy()
    e = xyz[:, 1:4] - xyz[:, 0:1]
    neg = np.einsum("kd,kd->k", np.cross(e[:, 0], e[:, 1]), e[:, 2]) < 0
    P[neg] = P[neg][:, [0, 2, 1, 3]]
    r, s, t = rst[:, 0], rst[:, 1], rst[:, 2]
    lam = np.stack([-(1 + r + s + t) / 2, (1 + r) / 2, (1 + s) / 2, (1 + t) / 2], axis=1)
    return np.ascontiguousarray(m["phi"](np.einsum("iv,kvd->kid", lam, P)))


def sphere_domain_map(m, s0=None, tol=1e-9):
    """Map for the trumpet's spherical domain (trumpet_domain('sphere')):
    its outer side vertices lie on the sphere |p - c| = R about the x axis
    and its side faces are flat chords between them; the caps are planes
    x = const.  In the cross-section plane of a point p = (x, rho, theta)
    (cylindrical about the x axis), let rho_f be the radius at which the ray
    from the axis towards p meets the flat side boundary and rho_s(x) =
    sqrt(R^2 - (x - c_x)^2) the sphere's: p moves radially to
    rho (1 + w (rho_s / rho_f - 1)), w = smoothstep((rho/rho_f - s0)/(1 - s0)),
    which lays the side faces onto the sphere and the caps' rims onto circles
    (the caps stay planar) and leaves every point with rho < s0 rho_f in place.
    By default s0 = 1 - 0.75 d, d the largest relative radial depth
    1 - rho/rho_s of a vertex of an element with a face on the curved side:
    the blend stays inside the layer of boundary elements, so that mostly
    the elements at the boundary are curved.
    Returns m with 'param' (= xyz) and 'phi' added."""
    xyz, bc = m["xyz"], m["bc"]
    fv = np.array([(0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3)])
    k, f = np.nonzero(bc == BC_OUTFLOW_CHAR)
    tri = xyz[k[:, None], fv[f]]                                  # [nf, 3, 3]
    cand = tri[np.ptp(tri[..., 0], axis=1) > 0]                   # faces spanning two planes
    # the sphere (centre on the x axis): |p - c|^2 = R^2 on the side vertices
    # is linear in (c_x, R^2 - c_x^2)
    P = cand.reshape(-1, 3)
    A = np.stack([2 * P[:, 0], np.ones(len(P))], axis=1)
    b = np.sum(P * P, axis=1)
    sol = np.linalg.lstsq(A, b, rcond=None)[0]
    cx, R = float(sol[0]), float(np.sqrt(sol[1] + sol[0] ** 2))
    on = np.all(np.abs(np.linalg.norm(tri - np.array([cx, 0, 0]), axis=-1) - R) < 1e-7 * R, axis=1)
    side = tri[on & (np.ptp(tri[..., 0], axis=1) > 0)]           # flat side faces on the sphere
    x_lo, x_hi = side[..., 0].min(axis=1), side[..., 0].max(axis=1)
    if s0 is None:
        ks = k[on & (np.ptp(tri[..., 0], axis=1) > 0)]
        v = xyz[ks].reshape(-1, 3)
        rs = np.sqrt(np.maximum(R * R - (v[:, 0] - cx) ** 2, 1e-300))
        depth = float(np.max(1.0 - np.linalg.norm(v[:, 1:], axis=1) / rs))
        s0 = float(np.clip(1.0 - 0.75 * depth, 0.5, 0.95))

    def rho_flat(p):
        """Radius of the flat side boundary on the ray from the axis towards p."""
        out = np.full(len(p), np.inf)
        rho = np.linalg.norm(p[:, 1:], axis=1)
        d = np.zeros_like(p)
        d[:, 1:] = p[:, 1:] / rho[:, None]
        o = p.copy()
        o[:, 1:] = 0.0
        for j0 in range(0, len(side), 256):
            T = side[j0:j0 + 256]
            sel = (p[:, None, 0] >= x_lo[None, j0:j0 + 256] - tol) & \
                  (p[:, None, 0] <= x_hi[None, j0:j0 + 256] + tol)
            ii, jj = np.nonzero(sel)
            if len(ii) == 0:
                continue
            v0, e1, e2 = T[jj, 0], T[jj, 1] - T[jj, 0], T[jj, 2] - T[jj, 0]
            h = np.cross(d[ii], e2)
            a = np.einsum("nd,nd->n", e1, h)
            ok = np.abs(a) > 1e-14
            a = np.where(ok, a, 1.0)
            s = o[ii] - v0
            u = np.einsum("nd,nd->n", s, h) / a
            qv = np.cross(s, e1)
            v = np.einsum("nd,nd->n", d[ii], qv) / a
            t = np.einsum("nd,nd->n", e2, qv) / a
            hit = ok & (u >= -tol) & (v >= -tol) & (u + v <= 1 + tol) & (t > 0)
            np.minimum.at(out, ii[hit], t[hit])
        return out

    def phi(p):
        p = np.array(p, dtype=np.float64)
        flat = p.reshape(-1, 3)
        rho = np.linalg.norm(flat[:, 1:], axis=1)
        rho_s = np.sqrt(np.maximum(R * R - (flat[:, 0] - cx) ** 2, 0.0))
        near = rho > 0.95 * s0 * rho_s
        idx = np.nonzero(near)[0]
        if len(idx):
            rf = rho_flat(flat[idx])
            if not np.all(np.isfinite(rf)):
                raise ValueError("a point's ray misses the flat side boundary")
            w = _smoothstep((rho[idx] / rf - s0) / (1.0 - s0))
            flat[idx, 1:] *= (1.0 + w * (rho_s[idx] / rf - 1.0))[:, None]
        return flat.reshape(p.shape)

    out = dict(m)
    out["param"] = xyz.copy()
    out["phi"] = phi
    out["sphere"] = (np.array([cx, 0.0, 0.0]), R)
    out["blend_s0"] = s0
    return out
