"""Element order of a mesh: a Z-order (Morton) curve of the element
centroids, so that face neighbours lie close in memory.

An element order is a property of the mesh arrays, not of the method: each
element's right-hand side is the same arithmetic on the same neighbours in
any order, so a reordered mesh gives the same results, permuted.  Ordering
pays where the state outgrows the last-level cache and the neighbour traces
would otherwise be fetched from HBM.
"""
import numpy as np


def _spread3(x):
    """The low 21 bits of x with two zero bits after each (bit i -> 3 i)."""
    x = x.astype(np.uint64) & np.uint64(0x1FFFFF)
    for shift, mask in ((32, 0x1F00000000FFFF), (16, 0x1F0000FF0000FF), (8, 0x100F00F00F00F00F),
                        (4, 0x10C30C30C30C30C3), (2, 0x1249249249249249)):
        x = (x | (x << np.uint64(shift))) & np.uint64(mask)
    return x


def locality_order(m):
    """Permutation p of the elements of mesh m (arrays xyz [K, 4, 3], ...):
    element p[i] goes to position i, in Z-order of the centroids on a 2^21
    grid per axis (ties kept in generator order)."""
    c = np.asarray(m["xyz"], dtype=np.float64).mean(axis=1)
    lo = c.min(axis=0)
    span = float((c.max(axis=0) - lo).max()) or 1.0
    g = np.floor((c - lo) / span * (2 ** 21 - 1)).astype(np.int64)
    code = _spread3(g[:, 0]) | (_spread3(g[:, 1]) << np.uint64(1)) | (_spread3(g[:, 2]) << np.uint64(2))
    return np.argsort(code, kind="stable")


def reorder(m, p):
    """The mesh m with its elements in the order p: its xyz, EToV and bc
    arrays permuted (shared vertex ids unchanged)."""
    out = dict(m)
    for key in ("xyz", "EToV", "bc"):
        out[key] = np.asarray(m[key])[p]
    return out
