"""Probe location with curved elements (dg_probe_setup on a host-only context,
no GPU): on the box whose x = 1 face is bent onto a spherical cap, a point
between a boundary chord and the face bent outward over it, and points
between the straight and curved images of moved interior faces, land in an
element whose curved image holds them: that element's curved map, evaluated
with the returned weights, gives the point back, and the point's reference
coordinates lie in the reference tetrahedron.  Geometry only, so the checks
are exact up to rounding and need no oracle."""
import itertools

import numpy as np
import pytest

import paper_1710_03887_amd as dg
from workloads.curved import capped_box, curved_nodes


def _setup(N=3, n=3):
    m = capped_box(n)
    ctx = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], N, host_only=True)
    rst = dg.dg_reference_operators(ctx)["rst"]
    x = curved_nodes(m, rst)
    assert dg.dg_set_curved(ctx, x) > 0
    return m, ctx, rst, x


def _faces(m):
    """Every element face as (sorted vertex ids, element, local vertex triple)."""
    for k, ev in enumerate(m["EToV"]):
        for tri in itertools.combinations(range(4), 3):
            yield tuple(sorted(int(ev[i]) for i in tri)), k, tri


def _check_inside(ctx, rst, x, pts):
    el, w = dg.dg_probe_setup(ctx, pts, weights=True)
    for p, k, wk in zip(pts, el, w):
        # the element's curved map at the point's reference coordinates
        np.testing.assert_allclose(wk @ x[k], p, atol=1e-10)
        r, s, t = wk @ rst                      # linear functions are reproduced
        lam = (-(1 + r + s + t) / 2, (1 + r) / 2, (1 + s) / 2, (1 + t) / 2)
        assert min(lam) >= -1e-9, (k, lam)
    return el


def test_point_between_chord_and_bent_face():
    m, ctx, rst, x = _setup()
    phi, P = m["phi"], m["param"]                      # vertex pre-images [K, 4, 3]
    pts = []
    for key, k, tri in _faces(m):
        pv = P[k, list(tri)]
        if not np.all(np.abs(pv[:, 0] - 1.0) < 1e-12):
            continue                                    # a face on the cap
        S = m["xyz"][k, list(tri)].mean(axis=0)         # chord centroid
        C = phi(pv.mean(axis=0))                        # bent face over it
        assert C[0] > S[0] + 1e-3                       # the cap bulges outward
        pts.append(S + 0.5 * (C - S))
        if len(pts) == 4:
            break
    pts = np.array(pts)
    # outside the straight-sided mesh: without the curved set it is rejected
    ctx2 = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], 3, host_only=True)
    with pytest.raises(dg.DGError, match="outside the mesh"):
        dg.dg_probe_setup(ctx2, pts[:1])
    _check_inside(ctx, rst, x, pts)


def test_point_beyond_moved_interior_face():
    m, ctx, rst, x = _setup()
    phi, P = m["phi"], m["param"]
    owners = {}
    for key, k, tri in _faces(m):
        owners.setdefault(key, []).append((k, tri))
    moved = []
    for key, own in owners.items():
        if len(own) != 2:
            continue
        k, tri = own[0]
        S = m["xyz"][k, list(tri)].mean(axis=0)
        C = phi(P[k, list(tri)].mean(axis=0))
        if np.linalg.norm(C - S) > 1e-3:
            moved.append((np.linalg.norm(C - S), S, C))
    assert len(moved) >= 4
    moved.sort(key=lambda v: -v[0])
    # halfway between the straight and the curved image of the face: in the
    # straight image of one element and the curved image of the other
    pts = np.array([0.5 * (S + C) for _, S, C in moved[:6]])
    _check_inside(ctx, rst, x, pts)


def test_straight_elements_and_outside_points():
    m, ctx, rst, x = _setup()
    # centroids of straight elements (the map is the identity for x <= 0)
    # keep their element
    ks = np.flatnonzero((m["param"][:, :, 0] <= 0.0).all(axis=1))[:5]
    cen = m["xyz"][ks].mean(axis=1)
    el = _check_inside(ctx, rst, x, cen)
    np.testing.assert_array_equal(el, ks)
    with pytest.raises(dg.DGError, match="outside the mesh"):
        dg.dg_probe_setup(ctx, np.array([[1.5, 0.0, 0.0]]))
