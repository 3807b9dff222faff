"""Pins for the oracle's reference operators.

The mass and face-mass matrices are built from exact rational monomial
integrals; here they are checked against an independent Gauss-Jacobi
collapsed-coordinate quadrature (scipy), which integrates polynomials of the
needed degree exactly.  Differentiation is checked on every monomial, and
the three together through the discrete divergence theorem
  1^T M Dr u = sum_f (boundary integral of u n_r)  (reference normals).
"""
import numpy as np
import pytest
from scipy.special import roots_jacobi, roots_legendre

from oracle.operators import RefElement, monomial_exponents, FACE_PARAMS


def tet_quadrature(n):
    a, wa = roots_legendre(n)
    b, wb = roots_jacobi(n, 1.0, 0.0)
    c, wc = roots_jacobi(n, 2.0, 0.0)
    A, B, C = np.meshgrid(a, b, c, indexing="ij")
    W = wa[:, None, None] * wb[None, :, None] * wc[None, None, :] / 2.0 / 4.0
    t = C
    s = (1 + B) * (1 - C) / 2 - 1
    r = (1 + A) * (1 - B) * (1 - C) / 4 - 1
    return np.stack([r.ravel(), s.ravel(), t.ravel()], 1), W.ravel()


def tri_quadrature(n):
    a, wa = roots_legendre(n)
    b, wb = roots_jacobi(n, 1.0, 0.0)
    A, B = np.meshgrid(a, b, indexing="ij")
    W = wa[:, None] * wb[None, :] / 2.0
    u = (1 + A) * (1 - B) / 2 - 1
    return np.stack([u.ravel(), B.ravel()], 1), W.ravel()


def lagrange_eval(ref, pts):
    """Values of the nodal Lagrange basis at points: [npts, Np]."""
    exps = monomial_exponents(ref.N)
    P = np.stack([pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c for a, b, c in exps], 1)
    return P @ np.linalg.inv(ref.V)


def face_point(f, uv):
    """Reference coordinates of face-parameter points on face f."""
    u, v = uv[:, 0], uv[:, 1]
    m1 = -np.ones_like(u)
    if f == 0:
        return np.stack([u, v, m1], 1)
    if f == 1:
        return np.stack([u, m1, v], 1)
    if f == 2:
        return np.stack([-1 - u - v, u, v], 1)
    return np.stack([m1, u, v], 1)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_differentiation_exact_on_monomials(N):
    ref = RefElement(N)
    r, s, t = ref.rst.T
    for a, b, c in monomial_exponents(N):
        f = r ** a * s ** b * t ** c
        fr = a * r ** max(a - 1, 0) * s ** b * t ** c
        fs = b * r ** a * s ** max(b - 1, 0) * t ** c
        ft = c * r ** a * s ** b * t ** max(c - 1, 0)
        assert np.allclose(ref.Dr @ f, fr, atol=1e-11)
        assert np.allclose(ref.Ds @ f, fs, atol=1e-11)
        assert np.allclose(ref.Dt @ f, ft, atol=1e-11)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_mass_matrix_vs_gauss_jacobi(N):
    ref = RefElement(N)
    x, w = tet_quadrature(N + 2)
    L = lagrange_eval(ref, x)
    Mq = L.T @ (w[:, None] * L)
    assert np.allclose(ref.M, Mq, atol=1e-12)
    assert abs(ref.M.sum() - 4.0 / 3.0) < 1e-12


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_face_mass_vs_gauss_jacobi(N):
    ref = RefElement(N)
    uv, w = tri_quadrature(N + 2)
    for f in range(4):
        L = lagrange_eval(ref, face_point(f, uv))
        Eq = L.T @ (w[:, None] * L)                       # Np x Np on the face
        E = ref.Emass[f]                                  # Np x Nfp
        assert np.allclose(E, Eq[:, ref.Fmask[f]], atol=1e-12)
        assert abs(E.sum() - 2.0) < 1e-12
        assert np.allclose(ref.M @ ref.LIFT[:, f * ref.Nfp:(f + 1) * ref.Nfp], E, atol=1e-12)


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_discrete_divergence_theorem(N):
    """int_T du/dx_a = sum_f int_f u n_a, with reference outward normals
    scaled to face parameters: f0 (t=-1): n=-e_t; f1 (s=-1): -e_s;
    f2 (r+s+t=-1): (1,1,1) per unit parameter area; f3 (r=-1): -e_r."""
    ref = RefElement(N)
    rng = np.random.default_rng(0)
    u = rng.standard_normal(ref.Np)
    one = np.ones(ref.Np)
    nparam = np.array([[0, 0, -1], [0, -1, 0], [1, 1, 1], [-1, 0, 0]], dtype=float)
    for a, D in enumerate((ref.Dr, ref.Ds, ref.Dt)):
        lhs = one @ ref.M @ D @ u
        rhs = sum(nparam[f, a] * (ref.Emass[f].sum(axis=0) @ u[ref.Fmask[f]])
                  for f in range(4))
        assert abs(lhs - rhs) < 1e-11 * (1 + abs(lhs))


def _node_permutation(rst, sig):
    """Node permutation induced by the vertex permutation sig of the
    reference tetrahedron (vertices (-1,-1,-1), (1,-1,-1), (-1,1,-1),
    (-1,-1,1)): node n goes to the node whose barycentric coordinates are
    n's with vertex v's coordinate moved to vertex sig[v]; None if the node
    set is not mapped onto itself."""
    lam = np.stack([-(1 + rst.sum(1)) / 2, (1 + rst[:, 0]) / 2, (1 + rst[:, 1]) / 2,
                    (1 + rst[:, 2]) / 2], 1)
    tgt = np.empty_like(lam)
    tgt[:, list(sig)] = lam
    d = np.abs(tgt[:, None, :] - lam[None, :, :]).max(2)
    p = d.argmin(1)
    return p if (d[np.arange(len(p)), p] < 1e-12).all() else None


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_operators_follow_tetrahedron_symmetry(N):
    """The reference tetrahedron is mapped onto itself by its 24 vertex
    permutations (affine maps of unit determinant magnitude), the Warp &
    Blend node set with it (Section 2.1), so the operators are tied to each
    other: swapping vertices 2 and 3 swaps r and s, hence Ds(i, j) =
    Dr(p(i), p(j)) for the induced node permutation p (Dt likewise with
    vertices 2 and 4); and a permutation taking face f onto face 0 carries
    face f's LIFT columns onto face 0's.  A derivative taken along the wrong
    coordinate, a sign, or a face mask of the wrong face breaks these.  The
    face relation holds up to the rounding of the monomial construction
    (largest at N = 5, 3e-8 of max |LIFT|)."""
    ref = RefElement(N)
    perms = [_node_permutation(ref.rst, s) for s in __import__("itertools").permutations(range(4))]
    assert all(p is not None for p in perms)                  # the node set is symmetric
    for D, sig in ((ref.Ds, (0, 2, 1, 3)), (ref.Dt, (0, 3, 2, 1))):
        p = _node_permutation(ref.rst, sig)
        np.testing.assert_allclose(D, ref.Dr[np.ix_(p, p)], rtol=0, atol=1e-9 * np.abs(ref.Dr).max())
    Fm = np.asarray(ref.Fmask).reshape(4, ref.Nfp)
    on0 = -np.ones(ref.Np, int)
    on0[Fm[0]] = np.arange(ref.Nfp)
    L = ref.LIFT
    for f in range(4):
        best = np.inf
        for p in perms:
            t = on0[p[Fm[f]]]
            if (t >= 0).all():
                best = min(best, np.abs(L[:, f * ref.Nfp:(f + 1) * ref.Nfp] - L[p][:, t]).max())
        assert best <= 1e-7 * np.abs(L).max(), (f, best)
