"""Shared test helpers: oracle <-> library state conversion (node order and
perturbation form).  Test-only code; the library never imports it."""
import numpy as np

import paper_1710_03887_amd as dg
from oracle import euler
from oracle.mesh import Mesh
from oracle.operators import RefElement
from oracle.mesh import FACE_VERTS as _FACE_VERTS
from workloads import BC_INTERIOR as _BC_INTERIOR, BC_OUTFLOW_CHAR as _BC_OUTFLOW_CHAR

_REFS = {}


def ref_of(N):
    if N not in _REFS:
        _REFS[N] = RefElement(N)
    return _REFS[N]


def node_perm(ctx, ref):
    """perm with library node i == oracle node perm[i] (reference nodes)."""
    rst = dg.dg_reference_operators(ctx)["rst"]
    d = np.linalg.norm(rst[:, None] - ref.rst[None], axis=-1)
    perm = d.argmin(axis=1)
    assert d.min(axis=1).max() < 1e-12 and len(set(perm.tolist())) == ref.Np
    return perm


def phys_kwargs(phys):
    return dict(gamma=phys.gamma, rho0=phys.rho0, u0=tuple(phys.u0), p0=phys.p0,
                inflow_amp=phys.amp, inflow_alpha=phys.alpha)


class Pair:
    """A mesh set up on both sides."""

    def __init__(self, m, N, phys, precision=dg.DG_FP32):
        self.ref = ref_of(N)
        self.bc = np.asarray(m["bc"])
        self.mesh = Mesh(self.ref, m["xyz"], m["EToV"], m["bc"])
        self.phys = phys
        self.ctx = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], N, precision=precision,
                                    **phys_kwargs(phys))
        self.perm = node_perm(self.ctx, self.ref)

    def to_device(self, q_oracle):
        """Full FP64 oracle state [K,5,Np] -> device FP32 perturbation."""
        import torch
        qp = (q_oracle - self.phys.q0[None, :, None])[:, :, self.perm]
        return torch.tensor(qp, dtype=torch.float32, device="cuda").contiguous()

    def from_device(self, q_dev, perturbation=True):
        """Device FP32 state -> FP64 oracle layout (adds q0 back)."""
        x = q_dev.double().cpu().numpy()
        out = np.empty_like(x)
        out[:, :, self.perm] = x
        if perturbation:
            out += self.phys.q0[None, :, None]
        return out

    def rates_from_device(self, r_dev):
        return self.from_device(r_dev, perturbation=False)


def rel_l2(mesh, a, b):
    """Mass-matrix relative L2 of a - b against b, over all variables."""
    from oracle.norms import l2
    num = sum(l2(mesh, (a - b)[:, v]) ** 2 for v in range(a.shape[1]))
    den = sum(l2(mesh, b[:, v]) ** 2 for v in range(b.shape[1]))
    return float(np.sqrt(num / den))


# ---- element samples of large meshes ------------------------------------------

def face_keys(EToV):
    f = np.sort(EToV[:, np.array(_FACE_VERTS)], axis=2).astype(np.int64)   # [K, 4, 3]
    assert f.max() < (1 << 21)
    return (f[..., 0] << 42) | (f[..., 1] << 21) | f[..., 2]


def neighbour_patch(m, sample, keys):
    """Sample elements plus every element sharing a face with one of them;
    faces left unmatched inside the patch get the characteristic tag (they
    bound neighbours only, never a sampled element)."""
    touch = np.isin(keys, keys[sample].ravel()).any(axis=1)
    idx = np.union1d(sample, np.nonzero(touch)[0])
    bc = m["bc"][idx].copy()
    pk = keys[idx]
    uniq, counts = np.unique(pk.ravel(), return_counts=True)
    single = np.isin(pk, uniq[counts == 1])
    loose = single & (bc == _BC_INTERIOR)
    assert not np.isin(idx[np.nonzero(loose)[0]], sample).any()
    bc[loose] = _BC_OUTFLOW_CHAR
    return idx, {"xyz": m["xyz"][idx], "EToV": m["EToV"][idx], "bc": bc}


def oriented_nodes(xyz, lam):
    """Nodal coordinates [K, Np, 3] with the oracle's orientation rule
    (negatively oriented elements swap local vertices 1 and 2)."""
    e = xyz[:, 1:4] - xyz[:, 0:1]
    neg = np.einsum("kd,kd->k", np.cross(e[:, 0], e[:, 1]), e[:, 2]) < 0
    xyz = xyz.copy()
    xyz[neg] = xyz[neg][:, [0, 2, 1, 3]]
    return np.einsum("iv,kvd->kid", lam, xyz)


def rel_l2_rows(mesh, rows, a, b):
    """rel_l2 restricted to the elements `rows` of mesh (a, b: [len(rows), 5, Np])."""
    M, J = mesh.ref.M, mesh.J[rows]
    num = sum(np.sum(J * np.einsum("ki,ij,kj->k", a[:, v] - b[:, v], M, a[:, v] - b[:, v]))
              for v in range(5))
    den = sum(np.sum(J * np.einsum("ki,ij,kj->k", b[:, v], M, b[:, v])) for v in range(5))
    return float(np.sqrt(num / den))


# ---- node-by-node comparison ---------------------------------------------------

TAG_NAMES = {1: "char_outflow", 2: "pass_through", 3: "wall", 4: "inflow", 5: "learned"}
VAR_NAMES = ("rho", "rho_u", "rho_v", "rho_w", "E")
TILE = 16   # elements per tile of the library's stage kernel


def element_groups(bc, tile=TILE):
    """Element index sets that a localized defect would show up in: every
    element, elements whose four faces are interior, elements with a face of
    each boundary tag present, and the last tile of `tile` consecutive
    elements (partial when K is not a multiple of it)."""
    bc = np.asarray(bc)
    K = bc.shape[0]
    groups = {"all": np.arange(K)}
    inner = np.nonzero((bc == _BC_INTERIOR).all(axis=1))[0]
    if inner.size:
        groups["interior"] = inner
    for tag, name in TAG_NAMES.items():
        rows = np.nonzero((bc == tag).any(axis=1))[0]
        if rows.size:
            groups[name] = rows
    groups["last_tile"] = np.arange((K - 1) // tile * tile, K)
    return groups


def nodewise_errors(a, b, groups):
    """{group: [5]} max over the group's nodes of |a - b| per variable,
    relative to that variable's largest |b| over every element."""
    scale = np.abs(b).max(axis=(0, 2))
    scale = np.where(scale > 0, scale, 1.0)
    return {g: np.abs(a[rows] - b[rows]).max(axis=(0, 2)) / scale for g, rows in groups.items()}


def assert_nodewise(a, b, bc, bar, label=""):
    """Node-by-node parity: every variable at every node of every group
    within `bar` of the reference (relative to the variable's max |ref|).
    Prints the table; returns the largest error."""
    errs = nodewise_errors(a, b, element_groups(bc))
    worst = 0.0
    for g, e in errs.items():
        print(f"  {label} nodewise {g:>13s}: " + " ".join(f"{v}={x:.2e}" for v, x in
                                                          zip(VAR_NAMES, e)), flush=True)
        worst = max(worst, float(e.max()))
    bad = {g: float(e.max()) for g, e in errs.items() if not (e.max() < bar)}
    assert not bad, f"{label} nodewise error above {bar:g} in {bad}"
    return worst
