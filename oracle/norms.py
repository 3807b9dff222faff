"""Mass-matrix norms and conserved totals (oracle).

With the affine map, the integral of a nodal field e over element k is
J_k * 1^T M e_k and its squared L2 norm J_k * e_k^T M e_k (M the reference
mass matrix).
"""
import numpy as np

from .euler import primitive


def l2(mesh, e):
    """L2 norm of a nodal scalar field e [K, Np]."""
    M = mesh.ref.M
    return float(np.sqrt(np.sum(mesh.J * np.einsum("ki,ij,kj->k", e, M, e))))


def totals(mesh, q):
    """Integral of each conserved variable over the domain: [5]."""
    w = mesh.ref.M.sum(axis=0)                       # 1^T M
    return np.einsum("k,i,kvi->v", mesh.J, w, q)


def pressure(q, gamma):
    """Nodal pressure [K, Np] of a conserved state [K, 5, Np]."""
    return primitive(np.transpose(q, (0, 2, 1)), gamma)[..., 4]


def rel_l2_pressure(mesh, q_test, q_ref, phys):
    """|p_test - p_ref| / |p_ref - p0| in the mass-matrix L2 norm."""
    pt = pressure(q_test, phys.gamma)
    pr = pressure(q_ref, phys.gamma)
    return l2(mesh, pt - pr) / l2(mesh, pr - phys.p0)
