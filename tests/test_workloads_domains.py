"""The synthetic outer domains of the sensor study (Type A: box, sphere, cone,
spherical cone; Type B: half box, half cone): valid conforming meshes, the
circular domains' side vertices on their sphere / cone (the spherical cone's
on its cone or its cap sphere; the half cone's on the 45-degree cone
converging to its apex), and every sensor inside every domain."""
import numpy as np
import pytest

from oracle.mesh import Mesh
from oracle.operators import RefElement
from oracle import probes
from workloads import trumpet_domain, BC_OUTFLOW_CHAR
from workloads.trumpet import CONE_APEX_X, CONE_SLOPE, HALF_CONE_APEX_X
from paper_1710_03887_amd.sensors import SENSORS, sensor_points


@pytest.mark.parametrize("kind", ["box", "sphere", "cone", "scone", "half", "half-cone"])
def test_domain_mesh_and_sensors(kind):
    # the half cone's flat-faced side lies inside its circle by more than the
    # 2 cm that separate sensor 1 from it below about 14k tets
    m = trumpet_domain(kind, 15000 if kind == "half-cone" else 6000)
    mesh = Mesh(RefElement(1), m["xyz"], m["EToV"], m["bc"])
    k, f = np.nonzero((mesh.EToE < 0) & (mesh.bc == BC_OUTFLOW_CHAR))
    assert len(k) > 0
    if kind.endswith("cone") or kind == "sphere":
        fv = np.array([(0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3)])
        tri = mesh.xyz[k[:, None], fv[f]]
        side = np.ptp(tri[..., 0], axis=1) > 1e-12                 # faces spanning two planes
        v = tri[side].reshape(-1, 3)
        rho = np.linalg.norm(v[:, 1:], axis=1)
        if kind == "sphere":
            on = np.abs(np.linalg.norm(v - np.array([0.5, 0, 0]), axis=1) - 1.5) < 1e-9
        elif kind == "half-cone":
            on = np.abs(rho - (HALF_CONE_APEX_X - v[:, 0])) < 1e-9
        else:
            on = np.abs(rho - CONE_SLOPE * (v[:, 0] - CONE_APEX_X)) < 1e-9
            if kind == "scone":
                apex = np.array([CONE_APEX_X, 0.0, 0.0])
                on |= np.abs(np.linalg.norm(v - apex, axis=1) - (1.8 - CONE_APEX_X)) < 1e-9
        # the outer side faces: all their vertices on the surface (the
        # half domains' x = 1 plane also carries outflow faces)
        tri_on = on.reshape(-1, 3).all(axis=1)
        assert tri_on.sum() > 0.5 * side.sum()
    elem, _ = probes.locate(mesh, sensor_points(m))
    assert (elem >= 0).all(), (kind, elem)


def test_locality_order_brings_neighbours_close():
    """The Z-order of element centroids is a permutation that keeps every
    element and face tag, and brings face neighbours close in memory (the
    median index distance between neighbours falls at least tenfold from
    the generator's slice order)."""
    from workloads import locality_order, reorder
    m = trumpet_domain("box", 20_000)
    p = locality_order(m)
    assert np.array_equal(np.sort(p), np.arange(len(p)))
    r = reorder(m, p)
    ref = RefElement(1)
    dist = []
    for mm in (m, r):
        mesh = Mesh(ref, mm["xyz"], mm["EToV"], mm["bc"])
        k, f = np.nonzero(mesh.EToE >= 0)
        dist.append(np.median(np.abs(mesh.EToE[k, f] - k)))
        assert np.array_equal(np.bincount(np.ravel(mm["bc"])), np.bincount(np.ravel(m["bc"])))
    print(f"median neighbour index distance: {dist[0]:.0f} -> {dist[1]:.0f}")
    assert dist[1] * 10 <= dist[0]
