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
