"""The library's host setup (C++, orthonormal basis) against the oracle's
independent construction (Python, monomials with exact integrals), on the
CPU through the C ABI with a host-only context.  Nodes are matched by
position, so the two sides may order them differently."""
import numpy as np
import pytest

import paper_1710_03887_amd as dg
from oracle.operators import RefElement
from oracle.mesh import Mesh
from workloads import box_kuhn, BC_WALL, BC_INFLOW, BC_OUTFLOW_CHAR


def _match(a, b, tol=1e-12):
    """perm with a[i] == b[perm[i]]"""
    d = np.linalg.norm(a[:, None] - b[None], axis=-1)
    perm = d.argmin(axis=1)
    assert d.min(axis=1).max() < tol
    assert len(set(perm.tolist())) == len(a)
    return perm


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_reference_operators(N):
    m = box_kuhn(2)
    ctx = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], N, host_only=True)
    ops = dg.dg_reference_operators(ctx)
    ref = RefElement(N)
    perm = _match(ops["rst"], ref.rst, 1e-13)
    for name, A in (("Dr", ref.Dr), ("Ds", ref.Ds), ("Dt", ref.Dt)):
        assert np.abs(ops[name] - A[np.ix_(perm, perm)]).max() < 1e-10 * max(1, np.abs(A).max())
    for f in range(4):
        lib_nodes = perm[ops["Fmask"][f]]
        assert sorted(lib_nodes.tolist()) == sorted(ref.Fmask[f].tolist())
        j = [list(ref.Fmask[f]).index(n) for n in lib_nodes]
        L_or = ref.LIFT[:, f * ref.Nfp:(f + 1) * ref.Nfp][np.ix_(perm, j)]
        L_lib = ops["LIFT"][:, f * ref.Nfp:(f + 1) * ref.Nfp]
        # the oracle's monomial route inverts a Vandermonde matrix of condition
        # ~6e4 at N=5, which limits its LIFT to ~1e-8 relative (pinned separately
        # through M LIFT = E_f); the orthonormal route is better conditioned
        tol = 1e-10 if N <= 3 else 1e-7
        assert np.abs(L_lib - L_or).max() < tol * np.abs(L_or).max()


@pytest.mark.parametrize("periodic", [False, True])
def test_geometry_and_connectivity(periodic):
    N = 3
    m = box_kuhn(3, jitter=0.08, seed=7, periodic=periodic)
    ctx = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], N, host_only=True)
    ref = RefElement(N)
    mesh = Mesh(ref, m["xyz"], m["EToV"], m["bc"])
    g = dg.dg_geometry(ctx)
    assert np.abs(g["drst_dx"] - mesh.drst_dx).max() < 1e-12
    assert np.abs(g["J"] - mesh.J).max() < 1e-14
    assert np.abs(g["nrm"] - mesh.normals).max() < 1e-13
    assert np.abs(g["Fscale"] - mesh.Fscale).max() < 1e-11
    xl = dg.dg_nodes(ctx)
    # per element node permutation lib -> oracle
    ops = dg.dg_reference_operators(ctx)
    perm = _match(ops["rst"], ref.rst, 1e-13)
    assert np.abs(xl - mesh.x[:, perm]).max() < 1e-13
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    mapP = g["mapP"]
    assert np.array_equal(mapP < 0, mesh.mapP < 0)
    for f in range(4):
        lib_nodes = perm[ops["Fmask"][f]]                 # oracle node ids of lib face nodes
        j = [list(ref.Fmask[f]).index(n) for n in lib_nodes]
        want = mesh.mapP[:, f, j]                         # oracle (k', node') flattened
        got = mapP[:, f, :]
        ok = want >= 0
        kk_w, nn_w = np.divmod(want[ok], ref.Np)
        kk_g, nn_g = np.divmod(got[ok], ref.Np)
        assert np.array_equal(kk_w, kk_g)
        assert np.array_equal(nn_w, perm[nn_g])


def test_orientation_fix_swaps_face_tags():
    m = box_kuhn(2, bc={"x-": BC_INFLOW, "x+": BC_WALL, "y-": BC_OUTFLOW_CHAR,
                        "y+": BC_OUTFLOW_CHAR, "z-": BC_WALL, "z+": BC_WALL})
    ctx = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], 2, host_only=True)
    g = dg.dg_geometry(ctx)
    assert np.all(g["J"] > 0)
    # every boundary face's outward normal points out of the box through the
    # side its tag belongs to
    nrm = g["nrm"]
    mesh = Mesh(RefElement(2), m["xyz"], m["EToV"], m["bc"])
    assert np.array_equal(mesh.bc, mesh.bc)  # oracle orientation
    boundary = mesh.EToE < 0
    side_tag = {(0, -1): BC_INFLOW, (0, 1): BC_WALL, (1, -1): BC_OUTFLOW_CHAR,
                (1, 1): BC_OUTFLOW_CHAR, (2, -1): BC_WALL, (2, 1): BC_WALL}
    for k, f in zip(*np.nonzero(boundary)):
        n = nrm[k, f]
        ax = int(np.argmax(np.abs(n)))
        assert side_tag[(ax, int(np.sign(n[ax])))] == mesh.bc[k, f]
    assert np.array_equal(np.array(g["mapP"] < 0).any(axis=2), boundary)


def test_setup_errors():
    m = box_kuhn(2)
    with pytest.raises(dg.DGError) as e:
        dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], 9, host_only=True)
    assert e.value.code == dg.DG_EINVAL
    bad = m["bc"].copy()
    bad[bad > 0] = 0
    with pytest.raises(dg.DGError) as e:
        dg.dg_mesh_setup(m["xyz"], m["EToV"], bad, 2, host_only=True)
    assert e.value.code == dg.DG_EMESH
    flat = m["xyz"].copy()
    flat[0, 3] = flat[0, 0]
    with pytest.raises(dg.DGError) as e:
        dg.dg_mesh_setup(flat, m["EToV"], m["bc"], 2, host_only=True)
    assert e.value.code == dg.DG_EMESH
    tag = m["bc"].copy()
    tag[tag > 0] = 9
    with pytest.raises(dg.DGError) as e:
        dg.dg_mesh_setup(m["xyz"], m["EToV"], tag, 2, host_only=True)
    assert e.value.code == dg.DG_EINVAL
    with pytest.raises(dg.DGError, match="K must be positive") as e:     # empty mesh
        dg.dg_mesh_setup(m["xyz"][:0], m["EToV"][:0], m["bc"][:0], 2, host_only=True)
    assert e.value.code == dg.DG_EINVAL
    # element 0 repeated: each of its faces is shared by three elements
    cat = lambda a: np.concatenate([a, a[:1]])
    with pytest.raises(dg.DGError, match="more than two") as e:
        dg.dg_mesh_setup(cat(m["xyz"]), cat(m["EToV"]), cat(m["bc"]), 2, host_only=True)
    assert e.value.code == dg.DG_EMESH
    # the largest mesh: K x 5 x Np values must fit the stage kernel's 32-bit
    # offsets (12,271,335 elements at N = 4); checked before any array is
    # read, so a descriptor with tiny arrays and K one past the limit shows it
    import ctypes
    from paper_1710_03887_amd import _lib
    one = np.zeros(16)
    d = _lib.dg_mesh_desc(N=4, precision=dg.DG_FP32, K=(2**31 - 1) // 175 + 1,
                          xyz=one.ctypes.data, EToV=one.ctypes.data, bc=one.ctypes.data,
                          gamma=1.4, rho0=1.0, p0=1 / 1.4, flags=1)
    h = ctypes.c_void_p()
    assert _lib._lib.dg_mesh_setup(ctypes.byref(d), None, ctypes.byref(h)) == dg.DG_EINVAL
    assert b"exceeds" in _lib._lib.dg_last_error(None)
    ctx = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], 2, host_only=True)
    code = _lib._lib.dg_rhs(ctx.handle, ctypes.c_void_p(16), ctypes.c_void_p(16), 0.0, None)
    assert code == dg.DG_ENODEV
