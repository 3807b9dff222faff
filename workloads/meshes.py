"""Synthetic tetrahedral meshes with the scales of the paper's workloads.

The paper meshes a modified trumpet inside seven outer domains with GMSH
(Section 1.2, Table 1: about 1e5 to 2e5 tetrahedra).  Those meshes and the
trumpet profile are not available, so every workload here is a seeded,
structured hexahedral map whose hexes are cut into six tetrahedra (Kuhn /
Freudenthal split along the main diagonal, which keeps the triangulation
conforming across hexes).

Every generator returns a dict of plain arrays:

``xyz``   float64 [K, 4, 3]  coordinates of each element's four vertices
``EToV``  int64   [K, 4]     topological vertex ids (periodic images share ids)
``bc``    int8    [K, 4]     tag of local face f, faces numbered
                             f0={v0,v1,v2}, f1={v0,v1,v3}, f2={v1,v2,v3},
                             f3={v0,v2,v3}; 0 marks an interior face.

Element orientation is left as generated (half of the Kuhn tetrahedra have a
negative Jacobian); consumers are expected to fix it.  A face shared by two
elements whose both sides carry a non-interior tag is a zero-thickness wall
seen from both sides.
"""
import numpy as np

BC_INTERIOR = 0
BC_OUTFLOW_CHAR = 1
BC_PASSTHRU = 2
BC_WALL = 3
BC_INFLOW = 4
BC_LEARNED = 5

FACE_VERTS = ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))

# Kuhn split: one tetrahedron per ordering of the three axes, all sharing the
# hex diagonal from corner (0,0,0) to corner (1,1,1).
_KUHN_PATHS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def _kuhn_corners():
    """Corner offsets [6, 4, 3] (in hex-local 0/1 units) of the six tets."""
    out = np.zeros((6, 4, 3), dtype=np.int64)
    for t, path in enumerate(_KUHN_PATHS):
        c = np.zeros(3, dtype=np.int64)
        out[t, 0] = c
        for v, ax in enumerate(path):
            c = c.copy()
            c[ax] = 1
            out[t, v + 1] = c
    return out


def _split_hexes(corner_index):
    """Tets of a structured grid: corner_index [n0,n1,n2] hex origins ->
    integer grid indices [K, 4, 3]."""
    off = _kuhn_corners()                      # [6,4,3]
    base = corner_index.reshape(-1, 1, 1, 3)   # [H,1,1,3]
    return (base + off[None]).reshape(-1, 4, 3)


def box_kuhn(n, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0), jitter=0.0, seed=0,
             periodic=False, bc=BC_OUTFLOW_CHAR):
    """Box [lo, hi] split into n^3 hexes, 6 tets each.

    ``n`` is an int or a triple.  ``jitter`` is the fraction of the smallest
    hex size by which vertices move, uniformly in [-jitter*h, jitter*h]^3,
    drawn from numpy's PCG64(seed); in a non-periodic box only vertices off
    the boundary move (faces stay planar), in a periodic box every
    topological vertex moves and its periodic images move with it.
    ``periodic`` is a bool or a triple of bools.  ``bc`` is a tag for every
    boundary face or a dict keyed by 'x-','x+','y-','y+','z-','z+'.
    """
    n = np.broadcast_to(np.asarray(n, dtype=np.int64), (3,)).copy()
    per = np.broadcast_to(np.asarray(periodic, dtype=bool), (3,)).copy()
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    h = (hi - lo) / n

    grid = np.stack(np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]),
                                indexing="ij"), axis=-1)
    gidx = _split_hexes(grid)                  # [K,4,3] grid indices 0..n
    K = gidx.shape[0]

    # topological ids: wrap periodic axes
    tidx = gidx.copy()
    for a in range(3):
        if per[a]:
            tidx[..., a] %= n[a]
    nv = n + 1
    EToV = (tidx[..., 0] * nv[1] + tidx[..., 1]) * nv[2] + tidx[..., 2]

    xyz = lo + gidx * h
    if jitter:
        rng = np.random.Generator(np.random.PCG64(seed))
        disp = rng.uniform(-1.0, 1.0, size=(int(np.prod(nv)), 3)) * (jitter * h.min())
        movable = np.ones(int(np.prod(nv)), dtype=bool)
        full = np.stack(np.meshgrid(np.arange(nv[0]), np.arange(nv[1]), np.arange(nv[2]),
                                    indexing="ij"), axis=-1).reshape(-1, 3)
        for a in range(3):
            if not per[a]:
                movable &= (full[:, a] > 0) & (full[:, a] < n[a])
        disp[~movable] = 0.0
        xyz = xyz + disp[EToV]

    tags = np.zeros((K, 4), dtype=np.int8)
    sides = {}
    for a, name in enumerate("xyz"):
        sides[name + "-"] = (a, 0)
        sides[name + "+"] = (a, None)
    for f, (i, j, k) in enumerate(FACE_VERTS):
        fv = gidx[:, [i, j, k], :]             # [K,3,3]
        for name, (a, at) in sides.items():
            if per[a]:
                continue
            pos = 0 if at == 0 else n[a]
            on = np.all(fv[:, :, a] == pos, axis=1)
            tag = bc[name] if isinstance(bc, dict) else bc
            tags[on, f] = tag
    return {"xyz": np.ascontiguousarray(xyz), "EToV": np.ascontiguousarray(EToV),
            "bc": tags}


def trumpet_domain(*args, **kwargs):  # defined in trumpet.py, re-exported here
    from .trumpet import trumpet_domain as _t
    return _t(*args, **kwargs)
