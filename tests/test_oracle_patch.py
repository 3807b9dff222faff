"""The sampled-patch evaluation used at full mesh sizes reproduces the
oracle's whole-mesh right-hand side exactly on the sampled elements: a
trumpet mesh (every boundary kind), N = 2, 300 random elements plus 50
touching each boundary kind; also the nodal coordinates built per element
chunk equal the oracle mesh's."""
import numpy as np

from oracle import euler
from oracle.mesh import Mesh
from oracle.nodes import barycentric
from workloads import trumpet_domain, gaussian_pulse, BC_WALL, BC_INFLOW, BC_OUTFLOW_CHAR
from helpers import ref_of, face_keys, neighbour_patch, oriented_nodes, rel_l2_rows


def _state(x, phys):
    prim = gaussian_pulse(x, 0.05 * phys.p0, 0.2, (0.85, 0.05, 0.0), phys.rho0, phys.p0,
                          phys.gamma)
    prim[..., 2] += 0.02 * np.exp(-((x[..., 0] - 1.2) ** 2) / 0.3)
    return euler.initial_state(prim, phys.gamma)


def test_patch_rhs_equals_full_rhs():
    m = trumpet_domain("box", 6000)
    K = m["EToV"].shape[0]
    ref = ref_of(2)
    phys = euler.Physics(amp=0.1 / 1.4, alpha=2 * np.pi * 565.0 / 343.0)
    full = Mesh(ref, m["xyz"], m["EToV"], m["bc"])
    assert np.array_equal(oriented_nodes(m["xyz"], barycentric(ref.rst)), full.x)
    rng = np.random.default_rng(1)
    sample = [rng.choice(K, 300, replace=False)]
    for tag in (BC_WALL, BC_INFLOW, BC_OUTFLOW_CHAR):
        cand = np.nonzero((m["bc"] == tag).any(axis=1))[0]
        sample.append(rng.choice(cand, min(50, cand.size), replace=False))
    sample = np.unique(np.concatenate(sample))
    idx, pm = neighbour_patch(m, sample, face_keys(m["EToV"]))
    assert sample.size < idx.size < K
    pmesh = Mesh(ref, pm["xyz"], pm["EToV"], pm["bc"])
    rows = np.searchsorted(idx, sample)
    t = 0.3
    r_full = euler.rhs(full, _state(full.x, phys), t, phys)[sample]
    r_patch = euler.rhs(pmesh, _state(pmesh.x, phys), t, phys)[rows]
    assert np.array_equal(r_full, r_patch)
    assert rel_l2_rows(pmesh, rows, r_patch, r_full) == 0.0
