"""Pins of the curved-element oracle against what geometry and the straight
scheme fix, independently of its own formulas:

* straight node positions reproduce the straight-sided geometry and
  right-hand side (the curved formulas reduce to the affine ones);
* on a box with one face bent onto a spherical cap, the curved elements'
  volume and cap area approach their values by adaptive quadrature far
  better than the flat mesh's, and the normals on the cap approach the
  sphere's radial direction;
* the chain-rule gradient at nodes equals a finite difference of the nodal
  interpolant through the numerically inverted element map, and face
  normals / Fscale equal the cross product of finite-difference surface
  tangents over a finite-difference Jacobian;
* shared face nodes coincide, a uniform (moving) state has zero right-hand
  side, and the right-hand side of a small acoustic plane wave converges to
  its exact time derivative with the order.
"""
import numpy as np
import pytest

from oracle import euler, curved
from oracle.mesh import Mesh, FACE_VERTS
from oracle.operators import RefElement, vandermonde
from workloads import box_kuhn, BC_OUTFLOW_CHAR, BC_WALL, BC_INFLOW, BC_PASSTHRU, plane_wave
from workloads.curved import capped_box, curved_nodes

_REF = {}


def ref_of(N):
    if N not in _REF:
        _REF[N] = RefElement(N)
    return _REF[N]


CAP_BC = {"x-": BC_WALL, "x+": BC_OUTFLOW_CHAR, "y-": BC_WALL, "y+": BC_WALL,
          "z-": BC_WALL, "z+": BC_WALL}


def capped(N, n=3, x0=0.0, bc=CAP_BC):
    m = capped_box(n, x0=x0, bc=bc)
    mesh = Mesh(ref_of(N), m["xyz"], m["EToV"], m["bc"])
    return m, mesh, curved.CurvedGeometry(mesh, curved_nodes(m, mesh.ref.rst))


def test_straight_nodes_reduce_to_affine():
    N = 3
    bc = {"x-": BC_INFLOW, "x+": BC_OUTFLOW_CHAR, "y-": BC_WALL, "y+": BC_PASSTHRU,
          "z-": BC_OUTFLOW_CHAR, "z+": BC_OUTFLOW_CHAR}
    m = box_kuhn((3, 2, 2), jitter=0.1, seed=4, bc=bc)
    mesh = Mesh(ref_of(N), m["xyz"], m["EToV"], m["bc"])
    geo = curved.CurvedGeometry(mesh, mesh.x)
    assert np.abs(geo.drst_dx - mesh.drst_dx[:, None]).max() < 1e-11 * np.abs(mesh.drst_dx).max()
    assert np.abs(geo.J / mesh.J[:, None] - 1).max() < 1e-12
    assert np.abs(geo.normals - mesh.normals[:, :, None]).max() < 1e-12
    assert np.abs(geo.Fscale / mesh.Fscale[:, :, None] - 1).max() < 1e-12
    phys = euler.Physics(u0=(0.05, -0.02, 0.01), amp=0.05 / 1.4, alpha=10.0)
    rng = np.random.Generator(np.random.PCG64(3))
    prim = np.empty((mesh.K, mesh.ref.Np, 5))
    prim[..., 0] = 1.0 + 0.02 * rng.standard_normal(prim.shape[:2])
    prim[..., 1:4] = np.array(phys.u0) + 0.02 * rng.standard_normal(prim.shape[:2] + (3,))
    prim[..., 4] = phys.p0 * (1 + 0.02 * rng.standard_normal(prim.shape[:2]))
    q = euler.initial_state(prim, phys.gamma)
    a = curved.rhs(mesh, geo, q, 0.1, phys)
    b = euler.rhs(mesh, q, 0.1, phys)
    assert np.abs(a - b).max() < 1e-11 * np.abs(b).max()


def _volume(mesh, J):
    w = mesh.ref.M.sum(axis=0)                        # integral of each basis function
    return float(np.sum(J * w[None, :]))


def _cap_area(mesh, Fscale, J):
    ref = mesh.ref
    tot = 0.0
    for f in range(4):
        w = ref.Emass[f][ref.Fmask[f]].sum(axis=0)    # face integral of each face basis function
        on = (mesh.EToE[:, f] < 0) & (mesh.bc[:, f] == BC_OUTFLOW_CHAR)
        sJ = Fscale[on, f] * J[on][:, ref.Fmask[f]]
        tot += float(np.sum(sJ * w[None, :]))
    return tot


def test_cap_volume_area_and_normals():
    from scipy.integrate import dblquad
    m = capped_box(1)
    c, R = m["sphere"]
    height = lambda z, y: c[0] + np.sqrt(R * R - y * y - z * z) + 1.0
    vol = dblquad(height, -1, 1, -1, 1, epsabs=1e-13, epsrel=1e-13)[0]
    area = dblquad(lambda z, y: R / np.sqrt(R * R - y * y - z * z), -1, 1, -1, 1,
                   epsabs=1e-13, epsrel=1e-13)[0]
    errs = []
    for N in (2, 3, 4):
        m, mesh, geo = capped(N)
        Jf = np.broadcast_to(mesh.J[:, None], geo.J.shape)
        ev = (abs(_volume(mesh, Jf) / vol - 1), abs(_volume(mesh, geo.J) / vol - 1))
        ea = (abs(_cap_area(mesh, np.broadcast_to(mesh.Fscale[:, :, None], geo.Fscale.shape), Jf) / area - 1),
              abs(_cap_area(mesh, geo.Fscale, geo.J) / area - 1))
        # normals on the cap against the sphere's radial direction
        ref = mesh.ref
        dev_c, dev_f = 0.0, 0.0
        for f in range(4):
            on = (mesh.EToE[:, f] < 0) & (mesh.bc[:, f] == BC_OUTFLOW_CHAR)
            if not on.any():
                continue
            xf = geo.x[on][:, ref.Fmask[f]]
            assert np.abs(np.linalg.norm(xf - c, axis=-1) - R).max() < 1e-13   # nodes on the sphere
            radial = (xf - c) / R
            dev_c = max(dev_c, float(np.abs(1 - np.sum(geo.normals[on, f] * radial, -1)).max()))
            dev_f = max(dev_f, float(np.abs(1 - np.sum(mesh.normals[on, f][:, None] * radial, -1)).max()))
        print(f"N={N}: volume err flat {ev[0]:.2e} curved {ev[1]:.2e}; cap area err flat {ea[0]:.2e} "
              f"curved {ea[1]:.2e}; 1-cos(normal, radial) flat {dev_f:.2e} curved {dev_c:.2e}")
        assert ev[1] < ev[0] / 20 and ea[1] < ea[0] / 20 and dev_c < dev_f / 5
        errs.append((ev[1], ea[1]))
    assert errs[2][0] < errs[0][0] and errs[2][1] < errs[0][1]


def _interp(ref, xe, r):
    """Element map and a nodal field at reference points r [n, 3]."""
    V = vandermonde(ref.N, np.atleast_2d(r))[0]
    return V @ np.linalg.inv(ref.V)


def _invert(ref, xe, x, r0):
    """Reference point of physical x in the element with node positions xe."""
    Vinv = np.linalg.inv(ref.V)
    r = np.array(r0, dtype=np.float64)
    for _ in range(50):
        V, Vr, Vs, Vt = vandermonde(ref.N, r[None])
        res = (V @ Vinv @ xe)[0] - x
        Jm = np.stack([(Vr @ Vinv @ xe)[0], (Vs @ Vinv @ xe)[0], (Vt @ Vinv @ xe)[0]], axis=1)
        dr = np.linalg.solve(Jm, res)
        r -= dr
        if np.abs(dr).max() < 1e-15:
            break
    return r


def test_gradient_matches_finite_differences():
    N = 3
    m, mesh, geo = capped(N, n=2)
    ref = mesh.ref
    rng = np.random.Generator(np.random.PCG64(8))
    ks = np.argsort(-np.abs(geo.J / mesh.J[:, None] - 1).max(axis=1))[:3]   # most curved
    h = 1e-5
    for k in ks:
        xe = geo.x[k]
        u = rng.standard_normal(ref.Np)
        grad = np.einsum("iad,ai->id", geo.drst_dx[k], np.stack([ref.Dr @ u, ref.Ds @ u, ref.Dt @ u]))
        for i in (0, ref.Np // 2, ref.Np - 1):
            fd = np.empty(3)
            for d in range(3):
                vals = []
                for sgn in (1, -1):
                    x = xe[i].copy()
                    x[d] += sgn * h
                    r = _invert(ref, xe, x, ref.rst[i])
                    vals.append((_interp(ref, xe, r[None]) @ u)[0])
                fd[d] = (vals[0] - vals[1]) / (2 * h)
            assert np.abs(grad[i] - fd).max() < 1e-6 * max(1.0, np.abs(fd).max()), (k, i, grad[i], fd)


# reference face coordinates: face f is parametrized by two of (r, s, t),
# the remaining one fixed (faces 0, 1, 3) or given by r = -1 - s - t (face 2)
def _face_point(f, u, v):
    if f == 0:
        return np.array([u, v, -1.0])
    if f == 1:
        return np.array([u, -1.0, v])
    if f == 2:
        return np.array([-1.0 - u - v, u, v])
    return np.array([-1.0, u, v])


def test_face_normals_match_surface_tangents():
    N = 3
    m, mesh, geo = capped(N, n=2)
    ref = mesh.ref
    ks = np.argsort(-np.abs(geo.J / mesh.J[:, None] - 1).max(axis=1))[:2]
    h = 1e-6
    uv_index = {0: (0, 1), 1: (0, 2), 2: (1, 2), 3: (1, 2)}
    for k in ks:
        xe = geo.x[k]
        centroid = xe.mean(axis=0)
        for f in range(4):
            for ii in (0, ref.Nfp - 1):
                node = ref.Fmask[f][ii]
                a, b = uv_index[f]
                u, v = ref.rst[node][a], ref.rst[node][b]
                X = lambda uu, vv: (_interp(ref, xe, _face_point(f, uu, vv)[None]) @ xe)[0]
                tu = (X(u + h, v) - X(u - h, v)) / (2 * h)
                tv = (X(u, v + h) - X(u, v - h)) / (2 * h)
                c = np.cross(tu, tv)
                if np.dot(c, X(u, v) - centroid) < 0:
                    c = -c
                r0 = ref.rst[node]
                Jm = np.stack([(_interp(ref, xe, (r0 + h * e)[None]) @ xe)[0]
                               - (_interp(ref, xe, (r0 - h * e)[None]) @ xe)[0]
                               for e in np.eye(3)], axis=1) / (2 * h)
                sJ, J = np.linalg.norm(c), np.linalg.det(Jm)
                assert np.abs(geo.normals[k, f, ii] - c / sJ).max() < 1e-7
                assert abs(geo.Fscale[k, f, ii] / (sJ / J) - 1) < 1e-7
                assert abs(geo.J[k, node] / J - 1) < 1e-7


def test_shared_face_nodes_coincide():
    m, mesh, geo = capped(4)
    inner = mesh.mapP >= 0
    xf = geo.x[:, mesh.ref.Fmask][inner]
    xp = geo.x.reshape(-1, 3)[mesh.mapP[inner]]
    assert np.abs(xf - xp).max() < 1e-14
    # the face normals of the two sides are opposite
    K, Nfp = mesh.K, mesh.ref.Nfp
    flatn = geo.normals.reshape(K * 4 * Nfp, 3)
    # the neighbour's normal at the same point: its face index from EToF, node from mapP
    for k in range(0, K, 37):
        for f in range(4):
            k2, f2 = mesh.EToE[k, f], mesh.EToF[k, f]
            if k2 < 0:
                continue
            for i in range(Nfp):
                node2 = mesh.mapP[k, f, i] - k2 * mesh.ref.Np
                j = int(np.nonzero(mesh.ref.Fmask[f2] == node2)[0][0])
                assert np.abs(geo.normals[k, f, i] + geo.normals[k2, f2, j]).max() < 1e-12
                assert abs(geo.Fscale[k, f, i] * geo.J[k, mesh.ref.Fmask[f][i]]
                           / (geo.Fscale[k2, f2, j] * geo.J[k2, node2]) - 1) < 1e-12


def test_uniform_moving_state_is_steady():
    phys = euler.Physics(u0=(0.1, -0.05, 0.03))
    for tag in (BC_PASSTHRU, BC_OUTFLOW_CHAR):
        m, mesh, geo = capped(3, bc=tag)
        q = np.broadcast_to(phys.q0[None, :, None], (mesh.K, 5, mesh.ref.Np)).copy()
        assert np.abs(curved.rhs(mesh, geo, q, 0.0, phys)).max() < 1e-12


def test_plane_wave_rhs_converges():
    """d q / dt of a small plane wave (exact for the linearized equations;
    the nonlinear remainder is of order amp^2) on the curved elements away
    from the boundary (where the characteristic ghost is not exact for
    oblique waves): it converges with the order, while the straight-sided
    operator applied to the same curved nodes stalls."""
    phys = euler.Physics()
    amp, kwave, dirn = 1e-5, 1.0, np.array([0.6, 0.48, 0.64])
    errs, errs_flat = [], []
    for N in (2, 3, 4):
        m, mesh, geo = capped(N, n=4)
        wave = lambda t: euler.initial_state(
            plane_wave(geo.x, t, amp, dirn, kwave, phys.rho0, phys.p0, phys.gamma), phys.gamma)
        h = 1e-4
        exact = (wave(h) - wave(-h)) / (2 * h)
        q = wave(0.0)
        sel = np.all(mesh.EToE >= 0, axis=1) & (np.abs(geo.J / mesh.J[:, None] - 1).max(axis=1) > 1e-3)
        assert sel.sum() > 50
        scale = np.abs(exact[sel]).max()
        e = np.abs(curved.rhs(mesh, geo, q, 0.0, phys)[sel] - exact[sel]).max() / scale
        e_flat = np.abs(euler.rhs(mesh, q, 0.0, phys)[sel] - exact[sel]).max() / scale
        print(f"N={N}: plane-wave rhs error curved {e:.2e}, straight operator {e_flat:.2e}")
        errs.append(e)
        errs_flat.append(e_flat)
    assert errs[2] < errs[1] < errs[0] and errs[2] < 1e-2
    assert errs[2] < errs_flat[2] / 10


def test_sphere_domain_map():
    """The trumpet's spherical domain: side-face nodes land on the sphere,
    caps stay planar, shared face nodes coincide, Jacobians stay positive,
    and the curved side boundary's area approaches the closed-form area of
    the spherical zone between the cap planes, 2 pi R (x_hi - x_lo)."""
    from workloads import trumpet_domain
    from workloads.curved import sphere_domain_map
    m = sphere_domain_map(trumpet_domain("sphere", 6000))
    c, R = m["sphere"]
    N = 3
    mesh = Mesh(ref_of(N), m["xyz"], m["EToV"], m["bc"])
    geo = curved.CurvedGeometry(mesh, curved_nodes(m, mesh.ref.rst))
    ref = mesh.ref
    inner = mesh.mapP >= 0
    assert np.abs(geo.x[:, ref.Fmask][inner] - geo.x.reshape(-1, 3)[mesh.mapP[inner]]).max() < 1e-13
    x_lo, x_hi = m["xyz"][..., 0].min(), m["xyz"][..., 0].max()
    area_c = area_f = 0.0
    for f in range(4):
        on = (mesh.EToE[:, f] < 0) & (mesh.bc[:, f] == BC_OUTFLOW_CHAR)
        xf = geo.x[on][:, ref.Fmask[f]]
        side = np.ptp(xf[..., 0], axis=1) > 1e-12
        cap = ~side
        if side.any():
            assert np.abs(np.linalg.norm(xf[side] - c, axis=-1) - R).max() < 1e-12
        if cap.any():
            assert np.abs(xf[cap][..., 0] - xf[cap][..., :1, 0]).max() < 1e-12   # planar caps
        w = ref.Emass[f][ref.Fmask[f]].sum(axis=0)
        k = np.nonzero(on)[0][side]
        area_c += float(np.sum(geo.Fscale[k, f] * geo.J[k][:, ref.Fmask[f]] * w))
        area_f += float(np.sum(mesh.Fscale[k, f][:, None] * mesh.J[k][:, None] * w))
    zone = 2 * np.pi * R * (x_hi - x_lo)
    print(f"zone area: flat faces {area_f / zone - 1:.2e}, curved {area_c / zone - 1:.2e}")
    assert abs(area_c / zone - 1) < abs(area_f / zone - 1) / 15


def _curved_points(mesh, geo, rows, rng):
    """Images under the curved maps of random reference points well inside
    the elements `rows` (barycentric coordinates >= 0.15)."""
    ref = mesh.ref
    lam = rng.dirichlet(np.ones(4), size=len(rows)) * 0.4 + 0.15
    r0 = 2.0 * lam[:, 1:] - 1.0
    Vinv = np.linalg.inv(ref.V)
    pts = np.stack([(vandermonde(ref.N, r0[i][None])[0] @ Vinv @ geo.x[k])[0] for i, k in enumerate(rows)])
    return pts, r0


def test_locate_in_curved_elements():
    """Newton's inversion of a curved map recovers the reference point that
    the forward map sent to x, in the element the straight geometry names."""
    m, mesh, geo = capped(3, n=3)
    moved = np.abs(geo.x - mesh.x).max(axis=(1, 2)) > 1e-8
    rng = np.random.default_rng(5)
    rows = rng.choice(np.nonzero(moved)[0], 30, replace=False)
    pts, r0 = _curved_points(mesh, geo, rows, rng)
    elem, rst = curved.locate(mesh, geo, pts, moved)
    same = elem == rows
    assert same.sum() >= 25                     # a point near a face may fall to the neighbour
    assert np.abs(rst[same] - r0[same]).max() < 1e-10


def test_library_curved_probe_weights_match_oracle():
    """The library's host path (host-only context, no GPU): dg_set_curved
    keeps the curved set, dg_probe_setup inverts curved maps; same elements
    and weights node by node as the oracle."""
    import paper_1710_03887_amd as dg
    from helpers import node_perm
    from oracle import probes
    m, mesh, geo = capped(3, n=3)
    moved = np.abs(geo.x - mesh.x).max(axis=(1, 2)) > 1e-8
    ctx = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], 3, host_only=True)
    n = dg.dg_set_curved(ctx, curved_nodes(m, dg.dg_reference_operators(ctx)["rst"]))
    assert n == moved.sum()
    rng = np.random.default_rng(6)
    rows = np.concatenate([rng.choice(np.nonzero(moved)[0], 20, replace=False),
                           rng.choice(np.nonzero(~moved)[0], 10, replace=False)])
    pts, _ = _curved_points(mesh, geo, rows, rng)
    e_or, rst = curved.locate(mesh, geo, pts, moved)
    e_lib, w_lib = dg.dg_probe_setup(ctx, pts, weights=True)
    assert np.array_equal(e_lib, e_or)
    w_or = probes.weights(mesh.ref, rst)
    assert np.abs(w_lib - w_or[:, node_perm(ctx, mesh.ref)]).max() < 1e-10
    # without the curved set the straight-sided weights differ in curved elements
    dg.dg_set_curved(ctx, None)
    _, w_flat = dg.dg_probe_setup(ctx, pts, weights=True)
    assert np.abs(w_flat - w_lib)[np.isin(e_lib, np.nonzero(moved)[0])].max() > 1e-4


def test_library_curved_set_rejections_host_only():
    """dg_set_curved's checks on the host (no GPU): tol <= 0, node positions
    that differ on the two sides of a shared face, a node Jacobian <= 0, and
    a quadrature-scheme context; a rejected call leaves no curved set."""
    import paper_1710_03887_amd as dg
    m, mesh, geo = capped(2, n=2)
    ctx = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], 2, host_only=True)
    ops = dg.dg_reference_operators(ctx)
    x = curved_nodes(m, ops["rst"])
    assert dg.dg_set_curved(ctx, x) > 0
    with pytest.raises(dg.DGError):
        dg.dg_set_curved(ctx, x, tol=0.0)
    mapP = dg.dg_geometry(ctx)["mapP"]
    k, f = [(k, f) for k in range(ctx.K) for f in range(4) if mapP[k, f, 0] >= 0][0]
    bad = x.copy()
    bad[k, ops["Fmask"][f, -1]] += 1e-3
    with pytest.raises(dg.DGError, match="coincide"):
        dg.dg_set_curved(ctx, bad)
    bad = x.copy()
    bad[0] = bad[0][::-1]
    with pytest.raises(dg.DGError):
        dg.dg_set_curved(ctx, bad)
    # nothing kept after the rejection: probes use the straight-sided weights
    pts = mesh.x[:3].mean(axis=1)
    e, w = dg.dg_probe_setup(ctx, pts, weights=True)
    dg.dg_set_curved(ctx, None)
    e2, w2 = dg.dg_probe_setup(ctx, pts, weights=True)
    assert np.array_equal(e, e2) and np.abs(w - w2).max() == 0.0
    quad = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], 2, host_only=True, quadrature=True)
    with pytest.raises(dg.DGError):
        dg.dg_set_curved(quad, x)
