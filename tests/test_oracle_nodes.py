"""Pins for the oracle's node sets (warp-and-blend construction).

Independent facts used: the Gauss-Lobatto-Legendre points (roots of P_N'
from numpy's Legendre class, checked against their closed forms for small N),
the exact node sets at N = 2 and 3, and the symmetry of the construction
under every permutation of the tetrahedron's vertices.
"""
import itertools

import numpy as np
import pytest

from oracle.nodes import warp_blend_nodes, barycentric, lgl_points, n_nodes, ALPHA_OPT
from oracle.operators import vandermonde
from oracle.operators import face_masks

VERTS = np.array([[-1, -1, -1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=float)
EDGES = [(a, b) for a in range(4) for b in range(a + 1, 4)]


def _as_set(pts, decimals=12):
    return sorted(tuple(np.round(p, decimals) + 0.0) for p in pts)


def test_lgl_closed_forms():
    assert np.allclose(lgl_points(2), [-1, 0, 1], atol=1e-15)
    assert np.allclose(lgl_points(3), [-1, -1 / np.sqrt(5), 1 / np.sqrt(5), 1], atol=1e-15)
    assert np.allclose(lgl_points(4), [-1, -np.sqrt(3 / 7), 0, np.sqrt(3 / 7), 1], atol=1e-15)


@pytest.mark.parametrize("N", range(1, 8))
def test_count_inside_and_faces(N):
    rst = warp_blend_nodes(N)
    assert rst.shape == (n_nodes(N), 3)
    lam = barycentric(rst)
    assert lam.min() > -1e-13
    fm = face_masks(rst)
    assert fm.shape == (4, (N + 1) * (N + 2) // 2)
    # distinct nodes
    d = np.linalg.norm(rst[:, None] - rst[None], axis=-1) + np.eye(len(rst))
    assert d.min() > 1e-3


def test_exact_N2():
    rst = warp_blend_nodes(2)
    expect = list(VERTS) + [0.5 * (VERTS[a] + VERTS[b]) for a, b in EDGES]
    assert _as_set(rst) == _as_set(expect)


def test_exact_N3():
    rst = warp_blend_nodes(3)
    g = 1 / np.sqrt(5)
    expect = list(VERTS)
    for a, b in EDGES:
        for x in (-g, g):   # edge parameter x in [-1,1] from vertex a to b
            expect.append(0.5 * (1 - x) * VERTS[a] + 0.5 * (1 + x) * VERTS[b])
    for face in itertools.combinations(range(4), 3):
        expect.append(VERTS[list(face)].mean(axis=0))
    assert _as_set(rst) == _as_set(expect)


@pytest.mark.parametrize("N", range(1, 8))
def test_edges_are_lgl(N):
    rst = warp_blend_nodes(N)
    lam = barycentric(rst)
    for a, b in EDGES:
        others = [v for v in range(4) if v not in (a, b)]
        on = np.all(np.abs(lam[:, others]) < 1e-12, axis=1)
        x = np.sort(lam[on, b] - lam[on, a])
        assert np.allclose(x, lgl_points(N), atol=1e-13)


@pytest.mark.parametrize("N", range(1, 8))
def test_symmetric_under_vertex_permutations(N):
    lam = barycentric(warp_blend_nodes(N))
    base = _as_set(lam, 11)
    for perm in itertools.permutations(range(4)):
        assert _as_set(lam[:, list(perm)], 11) == base


def _lebesgue(N, alpha, M=40):
    """max over the order-M barycentric lattice of sum_i |l_i| for the
    order-N nodes with blend parameter alpha (l_i their Lagrange basis)."""
    X = warp_blend_nodes(N, alpha)
    Vinv = np.linalg.inv(vandermonde(N, X)[0])
    b = np.array([(M - i - j - k, i, j, k) for i in range(M + 1) for j in range(M + 1 - i)
                  for k in range(M + 1 - i - j)], dtype=np.float64) / M
    verts = np.array([[-1, -1, -1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    L = vandermonde(N, b @ verts)[0] @ Vinv
    return np.abs(L).sum(axis=1).max()


@pytest.mark.parametrize("N", [4, 5])
def test_blend_parameter_is_a_lebesgue_minimizer(N):
    """The blend parameter of each order was optimized for a small Lebesgue
    constant; a check of the tabulated value (and of the blend formula) that
    does not come from the table: it is a local minimizer of the constant
    over alpha +- 0.05 and +- 0.2 (at N = 4 the constant is flat there, to
    1e-4 relative), and the neighbouring orders' values -- an index off by
    one -- give a clearly larger constant."""
    a0 = ALPHA_OPT[N - 1]
    L0 = _lebesgue(N, a0)
    for da in (-0.2, -0.05, 0.05, 0.2):
        if a0 + da >= 0.0:
            assert L0 <= _lebesgue(N, a0 + da) * (1 + 1e-4), (N, da)
    for a in (ALPHA_OPT[N - 2], ALPHA_OPT[N]):
        if abs(a - a0) > 0.3:
            assert _lebesgue(N, a) > L0 * (1 + 2e-3), (N, a)
