"""Synthetic trumpet-in-a-domain meshes.

The paper places a modified trumpet (straight bore joined to a flared bell,
Section 1.2) in seven outer domains meshed with GMSH (Table 1: about 1e5 to
2e5 tetrahedra).  Its profile points are not available, so the instrument
here is a stand-in with the stated end radii: a bore of radius 0.05 on
x in [0, 0.7] and an exponential flare r = 0.05 exp(kappa (x - 0.7)) up to
the mouth radius 0.4 at x = 1 (kappa = ln 8 / 0.3).  The instrument walls
are zero-thickness slip walls; the mouthpiece disc at x = 0 is the inflow
face (Section 2.4) seen from the bore and a wall seen from behind; the outer
boundary is characteristic outflow.

Grid: a two-dimensional O-grid of the cross-section (a Cartesian inner
square, rings out to the instrument circle, then graded rings out to the
outer boundary), each quad cut into two triangles, extruded along x through
planes that include x = 0, 0.7 and 1.  Each triangular prism is cut into
three tetrahedra with every side-face diagonal running from the bottom
vertex of lower cross-section id to the top vertex of higher id; the choice
depends only on the shared edge, so the tetrahedral mesh is conforming.

Outer domains (Type A: the whole instrument inside; Type B: the bore plus
only the region x >= 1 in front of the bell, Section 3):
  'box'       [-0.5, 1.8] x [-1, 1]^2;
  'sphere'    radius 1.5 about (0.5, 0, 0), cut by the planes where its
              cross-section becomes narrower than the grid needs (flat caps);
  'cone'      x in [-0.5, 1.8] inside the cone of half-angle 30 degrees about
              the x axis with its apex at x = -1.3 (radius 0.46 at the back
              cap, 1.79 at the front cap);
  'scone'     the same cone closed in front by the sphere about its apex
              through (1.8, 0, 0) instead of a flat cap (a spherical cone; flat
              cap where the sphere becomes too narrow for the grid, x ~ 1.65);
  'half'      Type B: the box region in front of the bell;
  'half-cone' Type B: the cone of half-angle 45 degrees whose base is the bell
              plane x = 1 (radius 1.02 there) and whose apex is on the axis at
              x = 2.02, cut by a flat cap where its radius falls to 0.15
              (x = 1.87): its side meets the outgoing pulse at about 45 degrees.
`scale` grows the box-like outer domains linearly about (0.65, 0, 0) with the
instrument fixed.
"""
import numpy as np

from .meshes import BC_INTERIOR, BC_INFLOW, BC_OUTFLOW_CHAR, BC_WALL, FACE_VERTS

BORE_R = 0.05
BELL_X0, BELL_X1 = 0.7, 1.0
MOUTH_R = 0.4
KAPPA = np.log(MOUTH_R / BORE_R) / (BELL_X1 - BELL_X0)
CENTER_X = 0.65
CONE_APEX_X, CONE_SLOPE = -1.3, float(np.tan(np.pi / 6))
# Type B half cone: converging at 45 degrees from the bell plane to an apex on
# the axis; the mesh stops at a flat cap of radius HALF_CONE_CAP_R
HALF_CONE_APEX_X, HALF_CONE_CAP_R = 2.02, 0.15


def instrument_radius(x):
    x = np.asarray(x, dtype=np.float64)
    return np.where(x <= BELL_X0, BORE_R,
                    BORE_R * np.exp(KAPPA * (np.minimum(x, BELL_X1) - BELL_X0)))


def _outer_radius(x, cone):
    """Radius of a conical outer boundary at x: slope (x - apex), closed by the
    sphere of radius sphere_r about the apex when one is given."""
    x = np.asarray(x, dtype=np.float64)
    r = cone["slope"] * (x - cone["apex"])
    if cone["sphere_r"] is not None:
        r = np.minimum(r, np.sqrt(np.maximum(cone["sphere_r"] ** 2 - (x - cone["apex"]) ** 2, 0.0)))
    return r


def _contour_radius(x, x_lo, x_hi):
    """Radius of the grid circle that carries the instrument wall on [0, 1],
    relaxed outside it (there it is only a grid line)."""
    x = np.asarray(x, dtype=np.float64)
    r = instrument_radius(np.clip(x, 0.0, BELL_X1))
    behind = np.clip(x / min(x_lo, -1e-9), 0.0, 1.0)
    front = np.clip((x - BELL_X1) / max(x_hi - BELL_X1, 1e-9), 0.0, 1.0)
    r = r + (0.25 - BORE_R) * behind ** 2
    r = r + (0.6 - MOUTH_R) * front ** 2
    return r


def _graded(a, b, n, ratio=1.0):
    """n cells on [a, b]; the last cell is `ratio` times the first."""
    if abs(ratio - 1.0) < 1e-12 or n == 1:
        return np.linspace(a, b, n + 1)
    g = ratio ** (1.0 / (n - 1))
    w = g ** np.arange(n)
    return a + (b - a) * np.concatenate([[0.0], np.cumsum(w) / w.sum()])


def _o_grid(nt, nr1, nr2):
    """Topology of the cross-section O-grid.

    Returns (kind, coords, quads): per node a (block, u, v) description and
    the quads as node-index quadruples in counter-clockwise order.
      inner nodes:  ('in', i, j) for the (nt+1)^2 Cartesian inner square,
      ring nodes:   ('ring', a, r) for perimeter index a in [0, 4 nt) and
                    ring layer r in [1, nr1 + nr2] (layer 0 is the inner
                    square's perimeter).
    """
    nid = {}
    desc = []

    def add(key):
        if key not in nid:
            nid[key] = len(desc)
            desc.append(key)
        return nid[key]

    for i in range(nt + 1):
        for j in range(nt + 1):
            add(("in", i, j))
    # perimeter of the inner square, counter-clockwise from (nt, 0)
    per = []
    for j in range(nt):
        per.append(("in", nt, j))
    for i in range(nt, 0, -1):
        per.append(("in", i, nt))
    for j in range(nt, 0, -1):
        per.append(("in", 0, j))
    for i in range(0, nt):
        per.append(("in", i, 0))
    P = len(per)
    nr = nr1 + nr2
    ring = [[None] * (nr + 1) for _ in range(P)]
    for a in range(P):
        ring[a][0] = add(per[a])
        for r in range(1, nr + 1):
            ring[a][r] = add(("ring", a, r))
    quads = []
    for i in range(nt):
        for j in range(nt):
            quads.append((nid[("in", i, j)], nid[("in", i + 1, j)],
                          nid[("in", i + 1, j + 1)], nid[("in", i, j + 1)]))
    for a in range(P):
        b = (a + 1) % P
        for r in range(nr):
            quads.append((ring[a][r], ring[a][r + 1], ring[b][r + 1], ring[b][r]))
    return desc, per, np.array(quads, dtype=np.int64)


def _perimeter_points(nt):
    """Points of the inner square's perimeter on the unit square (max-norm 1)."""
    s = np.linspace(-1.0, 1.0, nt + 1)
    pts = []
    for j in range(nt):
        pts.append((1.0, s[j]))
    for i in range(nt, 0, -1):
        pts.append((s[i], 1.0))
    for j in range(nt, 0, -1):
        pts.append((-1.0, s[j]))
    for i in range(0, nt):
        pts.append((s[i], -1.0))
    return np.array(pts)


def trumpet_domain(kind="box", target_K=200_000, scale=1.0, wall_tag=BC_WALL,
                   inflow_tag=BC_INFLOW, outer_tag=BC_OUTFLOW_CHAR, return_info=False):
    """Trumpet inside an outer domain, about target_K tetrahedra.

    Returns {'xyz', 'EToV', 'bc'} (see meshes.py) and, with return_info,
    an 'info' dict with the grid sizes and the wall/inflow geometry.
    """
    if kind not in ("box", "sphere", "half", "cone", "scone", "half-cone"):
        raise ValueError("kind must be 'box', 'sphere', 'half', 'cone', 'scone' or 'half-cone'")
    halfk = kind in ("half", "half-cone")
    if kind == "sphere":
        x_lo, x_hi, half_w = 0.5 - 1.5, 0.5 + 1.5, 1.5
    else:
        x_lo, x_hi, half_w = -0.5, 1.8, 1.0
    x_lo = CENTER_X + (x_lo - CENTER_X) * scale
    x_hi = CENTER_X + (x_hi - CENTER_X) * scale
    half_w *= scale
    sph_c, sph_r = np.array([0.5, 0.0, 0.0]), 1.5 * scale
    cone = None
    if kind in ("cone", "scone"):
        apex = CENTER_X + (CONE_APEX_X - CENTER_X) * scale
        cone = {"apex": apex, "slope": CONE_SLOPE,
                "sphere_r": (x_hi - apex) if kind == "scone" else None}
    elif kind == "half-cone":
        x_hi = HALF_CONE_APEX_X - HALF_CONE_CAP_R
        cone = {"apex": HALF_CONE_APEX_X, "slope": -1.0, "sphere_r": None}

    def layout(s):
        nt = max(2, int(round(6 * s)))
        nr1 = max(1, int(round(2 * s)))
        nr2 = max(3, int(round((13 + 3 * np.log(max(scale, 1.0))) * s)))
        nback = max(2, int(round(6 * s * (1 + 0.5 * np.log(max(scale, 1.0))))))
        nbore = max(4, int(round(24 * s)))
        nbell = max(2, int(round(12 * s)))
        nfront = max(3, int(round(16 * s * (1 + 0.5 * np.log(max(scale, 1.0))))))
        xs = np.unique(np.concatenate([
            _graded(0.0, x_lo, nback, 3.0 * scale)[::-1],
            np.linspace(0.0, BELL_X0, nbore + 1),
            np.linspace(BELL_X0, BELL_X1, nbell + 1),
            _graded(BELL_X1, x_hi, nfront, 4.0 * scale)]))
        if kind == "sphere":
            xs = _sphere_planes(xs, x_lo, x_hi, sph_c, sph_r)
        if kind == "scone":
            keep = _outer_radius(xs, cone) > 1.6 * _contour_radius(xs, x_lo, x_hi)
            xs = xs[keep]
        return nt, nr1, nr2, xs

    def count(s):
        nt, nr1, nr2, xs = layout(s)
        nq = nt * nt + 4 * nt * (nr1 + nr2)
        K = 6 * nq * (len(xs) - 1)
        if halfk:
            # rough: bore interior for x < 1 plus everything in front
            front = np.sum(xs >= BELL_X1) - 1
            inner = nt * nt + 4 * nt * nr1
            K = 6 * (nq * max(front, 0) + inner * np.sum(xs[:-1] < BELL_X1))
        return K

    s = 1.0
    for _ in range(40):
        K = count(s)
        if abs(K / target_K - 1) < 0.04:
            break
        s *= (target_K / K) ** (1.0 / 3.0)
    nt, nr1, nr2, xs = layout(s)
    if halfk:
        xs = xs[xs >= 0.0]
    return _assemble(kind, nt, nr1, nr2, xs, x_lo, x_hi, half_w, sph_c, sph_r, wall_tag,
                     inflow_tag, outer_tag, return_info, scale, cone=cone)


def _assemble(kind, nt, nr1, nr2, xs, x_lo, x_hi, half_w, sph_c, sph_r, wall_tag, inflow_tag,
              outer_tag, return_info, scale, ext_rings=None, cone=None):
    """Tetrahedra of the extruded O-grid.  `ext_rings` (box only) appends
    rings beyond the outer square: a list of half-widths > half_w; `cone`
    (apex x, slope) gives a circular outer boundary of radius
    slope (x - apex x)."""
    n_ext = 0 if ext_rings is None else len(ext_rings)
    desc, per, quads = _o_grid(nt, nr1, nr2 + n_ext)
    nodes2 = len(desc)
    nr = nr1 + nr2
    perim = _perimeter_points(nt)
    alpha = 0.55

    # cross-section coordinates of every 2D node at each x plane
    nx = len(xs)
    Y = np.empty((nx, nodes2, 2))
    layer = np.zeros(nodes2, dtype=np.int64)    # 0 inner square, else ring layer
    for n, key in enumerate(desc):
        if key[0] == "ring":
            layer[n] = key[2]
    gam = np.concatenate([[0.0], ((np.arange(1, nr2 + 1) / nr2) ** 1.5)])
    for ix, x in enumerate(xs):
        R = float(_contour_radius(x, x_lo, x_hi))
        if kind == "sphere":
            outer_r = np.sqrt(max(sph_r ** 2 - (x - sph_c[0]) ** 2, 0.0))
        elif cone is not None:
            outer_r = float(_outer_radius(x, cone))
            if x > BELL_X1 + 1e-12:   # in front of the bell the grid circle is only a
                R = min(R, 0.5 * outer_r)  # grid line: it follows a converging outer wall
        for n, key in enumerate(desc):
            if key[0] == "in":
                u = -1.0 + 2.0 * key[1] / nt
                v = -1.0 + 2.0 * key[2] / nt
                Y[ix, n] = alpha * R * np.array([u, v])
                continue
            a, r = key[1], key[2]
            S = perim[a]
            C = R * S / np.linalg.norm(S)
            if r <= nr1:
                w = r / nr1
                Y[ix, n] = (1 - w) * alpha * R * S + w * C
            elif r > nr:
                Y[ix, n] = ext_rings[r - nr - 1] * S
            else:
                if kind == "sphere" or cone is not None:
                    O = outer_r * S / np.linalg.norm(S)
                else:
                    O = half_w * S
                Y[ix, n] = C + gam[r - nr1] * (O - C)

    # triangles: each quad cut along the diagonal from its lowest node id
    tris = []
    for q in quads:
        m = int(np.argmin(q))
        a, b, c, d = (q[(m + k) % 4] for k in range(4))
        tris.append((a, b, c))
        tris.append((a, c, d))
    tris = np.array(tris, dtype=np.int64)
    tri_layer_max = layer[tris].max(axis=1)
    tri_inside = tri_layer_max <= nr1          # inside the instrument circle

    # prisms -> 3 tets: order the triangle's ids ascending (a < b < c);
    # bottom plane l, top plane l+1 (ids + nodes2)
    tri_sorted = np.sort(tris, axis=1)
    A, B, C_ = tri_sorted[:, 0], tri_sorted[:, 1], tri_sorted[:, 2]
    tets, tet_layer, tet_tri = [], [], []
    for l in range(nx - 1):
        if kind in ("half", "half-cone") and xs[l] < BELL_X1 - 1e-12:
            sel = tri_inside
        else:
            sel = np.ones(len(tris), dtype=bool)
        o0, o1 = l * nodes2, (l + 1) * nodes2
        a, b, c = A[sel], B[sel], C_[sel]
        t1 = np.stack([a + o0, b + o0, c + o0, c + o1], 1)
        t2 = np.stack([a + o0, b + o0, b + o1, c + o1], 1)
        t3 = np.stack([a + o0, a + o1, b + o1, c + o1], 1)
        tt = np.concatenate([t1, t2, t3])
        tets.append(tt)
        tet_layer.append(np.full(len(tt), l))
        idx = np.nonzero(sel)[0]
        tet_tri.append(np.concatenate([idx, idx, idx]))
    EToV = np.concatenate(tets)
    tet_layer = np.concatenate(tet_layer)
    K = EToV.shape[0]
    plane = EToV // nodes2
    node2 = EToV % nodes2
    xyz = np.empty((K, 4, 3))
    xyz[..., 0] = xs[plane]
    xyz[..., 1:] = Y[plane, node2]

    tags = np.zeros((K, 4), dtype=np.int8)
    for f, vs in enumerate(FACE_VERTS):
        fpl = plane[:, list(vs)]
        fn = node2[:, list(vs)]
        fl = layer[fn]
        fx = xs[fpl]
        on_contour = np.all(fl == nr1, axis=1)
        in_x = np.all((fx >= -1e-12) & (fx <= BELL_X1 + 1e-12), axis=1)
        # a wall face lies on the contour and spans two planes (a side face)
        spans = fpl.min(axis=1) != fpl.max(axis=1)
        wall = on_contour & in_x & spans
        flat = fpl.min(axis=1) == fpl.max(axis=1)
        disc = flat & np.isclose(fx[:, 0], 0.0) & np.all(fl <= nr1, axis=1)
        from_bore = xs[tet_layer] >= -1e-12
        tags[wall, f] = wall_tag
        tags[disc & from_bore, f] = inflow_tag
        tags[disc & ~from_bore, f] = wall_tag
    keys = np.sort(EToV[:, FACE_VERTS], axis=2).reshape(-1, 3)
    _, inv, cnt = np.unique(keys, axis=0, return_inverse=True, return_counts=True)
    single = (cnt[inv.ravel()] == 1).reshape(K, 4)
    tags[single & (tags == BC_INTERIOR)] = outer_tag
    out = {"xyz": np.ascontiguousarray(xyz), "EToV": np.ascontiguousarray(EToV), "bc": tags}
    if return_info:
        out["info"] = {"nt": nt, "nr1": nr1, "nr2": nr2, "x_planes": xs,
                       "quads_2d": len(quads), "kind": kind, "scale": scale}
    return out


def _sphere_planes(xs, x_lo, x_hi, c, r):
    """Keep planes where the sphere's cross-section stays wider than the
    contour circle by a margin."""
    cs = np.sqrt(np.maximum(r ** 2 - (xs - c[0]) ** 2, 0.0))
    keep = cs > 1.6 * _contour_radius(xs, x_lo, x_hi)
    return xs[keep]


def _growing_cells(a, b, h0, growth):
    """Planes from a to b (either direction) whose cells start near h0 and
    grow by `growth` per cell, rescaled to end exactly at b."""
    L = abs(b - a)
    h, tot, cells = h0 * growth, 0.0, []
    while tot + h < L:
        cells.append(h)
        tot += h
        h *= growth
    cells.append(max(L - tot, 0.5 * cells[-1] if cells else L))
    w = np.array(cells) * (L / np.sum(cells))
    return a + np.sign(b - a) * np.concatenate([[0.0], np.cumsum(w)])


def trumpet_nested(target_K=50_000, scale=3.0, growth=1.25):
    """The trumpet in the box domain (about target_K tetrahedra) and the same
    scene in an outer box `scale` times larger about (0.65, 0, 0) that
    contains the smaller mesh element for element (same vertices in the same
    local order), so that solutions compare node by node.

    Beyond the small box, x-planes and square rings are added with cells
    growing geometrically by `growth` from the small box's outermost cells.
    Returns (big, small, emap): emap[k] is the big-mesh element of small-mesh
    element k.
    """
    small = trumpet_domain("box", target_K, return_info=True)
    info = small["info"]
    nt, nr1, nr2, xs = info["nt"], info["nr1"], info["nr2"], info["x_planes"]
    x_lo, x_hi, half_w = -0.5, 1.8, 1.0
    X_lo = CENTER_X + (x_lo - CENTER_X) * scale
    X_hi = CENTER_X + (x_hi - CENTER_X) * scale
    H = half_w * scale
    back = _growing_cells(x_lo, X_lo, xs[1] - xs[0], growth)[1:][::-1]
    front = _growing_cells(x_hi, X_hi, xs[-1] - xs[-2], growth)[1:]
    xs_big = np.concatenate([back, xs, front])
    rings = _growing_cells(half_w, H, xs[-1] - xs[-2], growth)[1:]
    big = _assemble("box", nt, nr1, nr2, xs_big, x_lo, x_hi, half_w, None, None, BC_WALL,
                    BC_INFLOW, BC_OUTFLOW_CHAR, False, scale, ext_rings=list(rings))
    # element map by vertex coordinates
    def keys(m):
        return np.round(m["xyz"].reshape(len(m["xyz"]), 12), 9)
    ks, kb = keys(small), keys(big)
    allk = np.concatenate([ks, kb])
    _, inv = np.unique(allk, axis=0, return_inverse=True)
    inv = inv.ravel()
    pos = np.full(inv.max() + 1, -1, dtype=np.int64)
    pos[inv[len(ks):]] = np.arange(len(kb))
    emap = pos[inv[:len(ks)]]
    if np.any(emap < 0):
        raise RuntimeError("small mesh is not nested in the big mesh")
    small.pop("info")
    return big, small, emap
