"""Interpolation nodes on the reference tetrahedron (oracle, FP64).

The reference tetrahedron has vertices V0=(-1,-1,-1), V1=(1,-1,-1),
V2=(-1,1,-1), V3=(-1,-1,1); the barycentric coordinates of a point (r,s,t)
are lam0=-(1+r+s+t)/2, lam1=(1+r)/2, lam2=(1+s)/2, lam3=(1+t)/2.

The paper's own solver uses a modal orthonormal basis with Gauss quadrature
(Appendix A); the nodal scheme here places its Np=(N+1)(N+2)(N+3)/6 nodes by
Warburton's explicit warp-and-blend construction ("An explicit construction
of interpolation nodes on the simplex", J. Eng. Math. 2006), restated here:

1. start from the equispaced barycentric lattice of order N;
2. on every edge, the 1D warp moves equispaced points onto the
   Gauss-Lobatto-Legendre (LGL) points;
3. on every face the three edge warps are blended into the face (each
   weighted by the product of the two barycentrics of its edge and a factor
   1+(alpha*lam_opposite)^2);
4. the face warps are blended into the interior with the factor
   lam_b lam_c lam_d / prod(lam_x + lam_a/2) * (1+(alpha*lam_a)^2), where
   lam_a is the barycentric of the vertex opposite the face;
5. points lying on an edge take the pure edge warp.

The blend parameter alpha is Warburton's optimized value per order.
"""
import numpy as np

# Warburton's optimized 3D blend parameters for N = 1..15.
ALPHA_OPT = (0.0, 0.0, 0.0, 0.1002, 1.1332, 1.5608, 1.3413, 1.2577, 1.1603,
             1.10153, 0.6080, 0.4523, 0.8856, 0.8717, 0.9655)

# Equilateral tetrahedron used for the construction; vertex i corresponds to
# the reference vertex Vi (same barycentric coordinate).
_SQ3 = np.sqrt(3.0)
_SQ6 = np.sqrt(6.0)
EQ_VERTS = np.array([[-1.0, -1.0 / _SQ3, -1.0 / _SQ6],
                     [1.0, -1.0 / _SQ3, -1.0 / _SQ6],
                     [0.0, 2.0 / _SQ3, -1.0 / _SQ6],
                     [0.0, 0.0, 3.0 / _SQ6]])

# Faces as (P, Q, R): base edge P->Q, apex R; the fourth vertex is opposite.
WARP_FACES = ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))


def n_nodes(N):
    return (N + 1) * (N + 2) * (N + 3) // 6


def n_face_nodes(N):
    return (N + 1) * (N + 2) // 2


def lgl_points(N):
    """Gauss-Lobatto-Legendre points on [-1,1], ascending: +-1 and the roots
    of P_N'."""
    if N == 1:
        return np.array([-1.0, 1.0])
    inner = np.polynomial.legendre.Legendre.basis(N).deriv().roots()
    return np.concatenate([[-1.0], np.sort(np.real(inner)), [1.0]])


def _edge_warp_scaled(N, x):
    """w(x) = [sum_i (x_i^LGL - x_i^eq) l_i^eq(x)] / (1 - x^2), with the
    division carried out exactly on the Lagrange polynomials (the endpoint
    displacements vanish, and each interior l_i carries the factor
    (x+1)(x-1))."""
    xeq = np.linspace(-1.0, 1.0, N + 1)
    d = lgl_points(N) - xeq
    w = np.zeros_like(x)
    for i in range(1, N):
        term = np.full_like(x, d[i] / (1.0 - xeq[i] ** 2))
        for j in range(1, N):
            if j != i:
                term = term * (x - xeq[j]) / (xeq[i] - xeq[j])
        w = w + term
    return w


def _face_shift(N, alpha, l1, l2, l3):
    """2D warp of an equilateral triangle with barycentrics (l1, l2, l3):
    l1 is the apex; edge 2-3 is the base, along the x axis."""
    # edge opposite l1 (base, direction 0 deg), opposite l2 (120 deg),
    # opposite l3 (240 deg)
    w1 = 4 * l2 * l3 * _edge_warp_scaled(N, l3 - l2) * (1 + (alpha * l1) ** 2)
    w2 = 4 * l1 * l3 * _edge_warp_scaled(N, l1 - l3) * (1 + (alpha * l2) ** 2)
    w3 = 4 * l1 * l2 * _edge_warp_scaled(N, l2 - l1) * (1 + (alpha * l3) ** 2)
    c120, s120 = np.cos(2 * np.pi / 3), np.sin(2 * np.pi / 3)
    c240, s240 = np.cos(4 * np.pi / 3), np.sin(4 * np.pi / 3)
    dx = w1 + c120 * w2 + c240 * w3
    dy = s120 * w2 + s240 * w3
    return dx, dy


def equispaced_barycentric(N):
    """All (lam0..lam3) = (i,j,k,l)/N with i+j+k+l = N, [Np, 4]."""
    pts = []
    for a in range(N + 1):
        for b in range(N + 1 - a):
            for c in range(N + 1 - a - b):
                pts.append((N - a - b - c, a, b, c))
    return np.array(pts, dtype=np.float64) / max(N, 1)


def warp_blend_nodes(N, alpha=None):
    """Reference coordinates [Np, 3] of the order-N warp-and-blend nodes
    (blend parameter alpha, by default the optimized value of the order)."""
    if N < 1:
        raise ValueError("N must be >= 1")
    if alpha is None:
        alpha = ALPHA_OPT[N - 1] if N <= len(ALPHA_OPT) else 1.0
    lam = equispaced_barycentric(N)
    X = lam @ EQ_VERTS
    shift = np.zeros_like(X)
    tol = 1e-10
    for (P, Q, R) in WARP_FACES:
        A = ({0, 1, 2, 3} - {P, Q, R}).pop()
        la = lam[:, A]
        l1, l2, l3 = lam[:, R], lam[:, P], lam[:, Q]
        t1 = EQ_VERTS[Q] - EQ_VERTS[P]
        t1 = t1 / np.linalg.norm(t1)
        t2 = EQ_VERTS[R] - 0.5 * (EQ_VERTS[P] + EQ_VERTS[Q])
        t2 = t2 / np.linalg.norm(t2)
        dx, dy = _face_shift(N, alpha, l1, l2, l3)
        blend = l1 * l2 * l3
        denom = (l1 + 0.5 * la) * (l2 + 0.5 * la) * (l3 + 0.5 * la)
        ok = denom > tol
        blend[ok] = (1 + (alpha * la[ok]) ** 2) * blend[ok] / denom[ok]
        shift += (blend * dx)[:, None] * t1 + (blend * dy)[:, None] * t2
        on_edge = (la < tol) & (((l1 > tol).astype(int) + (l2 > tol) + (l3 > tol)) < 3)
        shift[on_edge] = dx[on_edge, None] * t1 + dy[on_edge, None] * t2
    X = X + shift
    # back to reference coordinates: X = (E1+E2+E3-E0)/2 + [E1-E0, E2-E0, E3-E0]/2 (r,s,t)
    A = 0.5 * np.stack([EQ_VERTS[1] - EQ_VERTS[0], EQ_VERTS[2] - EQ_VERTS[0],
                        EQ_VERTS[3] - EQ_VERTS[0]], axis=1)
    b = X - 0.5 * (EQ_VERTS[1] + EQ_VERTS[2] + EQ_VERTS[3] - EQ_VERTS[0])
    rst = np.linalg.solve(A, b.T).T
    return rst


def barycentric(rst):
    """Barycentric coordinates [.., 4] of reference points [.., 3]."""
    r, s, t = rst[..., 0], rst[..., 1], rst[..., 2]
    return np.stack([-(1 + r + s + t) / 2, (1 + r) / 2, (1 + s) / 2, (1 + t) / 2], axis=-1)
