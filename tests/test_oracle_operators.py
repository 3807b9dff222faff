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
