"""Reference-element operators from monomials and exact integrals (oracle).

Appendix A writes the solution on each element as an expansion in Np basis
functions (Eq. 11) and tests the conservation law against them (Eq. 10).
In nodal form the same space is spanned by the Lagrange polynomials of the
nodes; here every operator is expressed through the monomial basis
r^a s^b t^c (a+b+c <= N):

* V[i, m]   = monomial m at node i; Vr, Vs, Vt its partial derivatives;
* Dr = Vr V^-1 (and Ds, Dt): nodal differentiation;
* M = V^-T Mmono V^-1 with Mmono[m, n] = integral over the reference
  tetrahedron of monomial m times monomial n, evaluated exactly in rational
  arithmetic from  int_simplex x^i y^j z^k = i! j! k! / (i+j+k+3)!;
* E_f, the face mass of face f in the face's own parameters (a reference
  triangle of area 2), from  int_triangle x^i y^j = i! j! / (i+j+2)!;
* LIFT_f = M^-1 E_f.
"""
from fractions import Fraction
from math import comb, factorial

import numpy as np

from .nodes import warp_blend_nodes, n_nodes, n_face_nodes

# Face f: the plane it lies on and the two reference coordinates that
# parametrize it.  f0: t=-1, f1: s=-1, f2: r+s+t=-1, f3: r=-1.
FACE_PARAMS = ((0, 1), (0, 2), (1, 2), (1, 2))


def monomial_exponents(N, dim=3):
    out = []
    if dim == 3:
        for a in range(N + 1):
            for b in range(N + 1 - a):
                for c in range(N + 1 - a - b):
                    out.append((a, b, c))
    else:
        for a in range(N + 1):
            for b in range(N + 1 - a):
                out.append((a, b))
    return out


def _shifted_power_coeffs(A):
    """(2x-1)^A = sum_i coef[i] x^i, exact."""
    return [Fraction(comb(A, i) * 2 ** i * (-1) ** (A - i)) for i in range(A + 1)]


def tet_monomial_integral(A, B, C):
    """Exact integral of r^A s^B t^C over the reference tetrahedron."""
    ca, cb, cc = _shifted_power_coeffs(A), _shifted_power_coeffs(B), _shifted_power_coeffs(C)
    total = Fraction(0)
    for i, a in enumerate(ca):
        for j, b in enumerate(cb):
            for k, c in enumerate(cc):
                total += a * b * c * Fraction(factorial(i) * factorial(j) * factorial(k),
                                              factorial(i + j + k + 3))
    return 8 * total


def tri_monomial_integral(A, B):
    """Exact integral of u^A v^B over the reference triangle
    {u,v >= -1, u+v <= 0} (area 2)."""
    ca, cb = _shifted_power_coeffs(A), _shifted_power_coeffs(B)
    total = Fraction(0)
    for i, a in enumerate(ca):
        for j, b in enumerate(cb):
            total += a * b * Fraction(factorial(i) * factorial(j), factorial(i + j + 2))
    return 4 * total


def vandermonde(N, rst):
    exps = monomial_exponents(N)
    r, s, t = rst[:, 0], rst[:, 1], rst[:, 2]
    V = np.stack([r ** a * s ** b * t ** c for (a, b, c) in exps], axis=1)

    def d(x, e):
        return e * x ** (e - 1) if e > 0 else np.zeros_like(x)
    Vr = np.stack([d(r, a) * s ** b * t ** c for (a, b, c) in exps], axis=1)
    Vs = np.stack([r ** a * d(s, b) * t ** c for (a, b, c) in exps], axis=1)
    Vt = np.stack([r ** a * s ** b * d(t, c) for (a, b, c) in exps], axis=1)
    return V, Vr, Vs, Vt


def face_masks(rst, tol=1e-10):
    r, s, t = rst[:, 0], rst[:, 1], rst[:, 2]
    tests = (np.abs(1 + t), np.abs(1 + s), np.abs(1 + r + s + t), np.abs(1 + r))
    return np.stack([np.nonzero(x < tol)[0] for x in tests])


class RefElement:
    """All reference operators for order N (FP64)."""

    def __init__(self, N):
        self.N = N
        self.Np = n_nodes(N)
        self.Nfp = n_face_nodes(N)
        self.rst = warp_blend_nodes(N)
        V, Vr, Vs, Vt = vandermonde(N, self.rst)
        Vinv = np.linalg.inv(V)
        self.V = V
        self.Dr = Vr @ Vinv
        self.Ds = Vs @ Vinv
        self.Dt = Vt @ Vinv
        exps = monomial_exponents(N)
        Mm = np.array([[float(tet_monomial_integral(a1 + a2, b1 + b2, c1 + c2))
                        for (a2, b2, c2) in exps] for (a1, b1, c1) in exps])
        self.M = Vinv.T @ Mm @ Vinv
        self.Minv = np.linalg.inv(self.M)
        self.Fmask = face_masks(self.rst)
        assert self.Fmask.shape == (4, self.Nfp)
        exps2 = monomial_exponents(N, dim=2)
        Mm2 = np.array([[float(tri_monomial_integral(a1 + a2, b1 + b2))
                         for (a2, b2) in exps2] for (a1, b1) in exps2])
        self.Emass = []          # per face: Np x Nfp
        self.LIFT = np.zeros((self.Np, 4 * self.Nfp))
        for f in range(4):
            uv = self.rst[self.Fmask[f]][:, FACE_PARAMS[f]]
            V2 = np.stack([uv[:, 0] ** a * uv[:, 1] ** b for (a, b) in exps2], axis=1)
            V2inv = np.linalg.inv(V2)
            M2 = V2inv.T @ Mm2 @ V2inv
            E = np.zeros((self.Np, self.Nfp))
            E[self.Fmask[f], :] = M2
            self.Emass.append(E)
            self.LIFT[:, f * self.Nfp:(f + 1) * self.Nfp] = self.Minv @ E
