"""The 100-step accuracy gates on the trumpet in the box reduced to 19,530
tetrahedra: the library's dg_run (its own time steps under CFL 0.5) against
the FP64 oracle's result stored in tests/golden/gate_<case>.npz by
tests/golden/make_gates.py, which calls the oracle alone.  Inputs are
tests/gate_cases.py.  Bars (relative L2 of the pressure perturbation,
mass-matrix norm, against the oracle's p - p0): FP32 1e-5, split-BF16 1e-3;
the end time must match the oracle's sum of time steps to 1e-6.

* N = 4 (the throughput workload's order): the inflow run from rest and the
  run with Gaussian pulses in the bell mouth and at the box's far face, in
  both forms;
* N = 5 (the precision workload's order): pulses of 0.5 %, 2 % and 10 % of
  p0, in both forms.
"""
import os

import numpy as np
import pytest

import paper_1710_03887_amd as dg
import gate_cases as gc
from oracle import euler, norms
from oracle.mesh import Mesh
from helpers import ref_of, node_perm, phys_kwargs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_MESH = {}


def _mesh(N):
    if N not in _MESH:
        m = gc.mesh()
        _MESH[N] = (m, Mesh(ref_of(N), m["xyz"], m["EToV"], m["bc"]))
    return _MESH[N]


SINGLE = [c for c in gc.CASES if not c.startswith("c4_")]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("case", SINGLE)
@pytest.mark.parametrize("form", ["fp32", "bf16"])
def test_gate_100_steps(case, form):
    spec = gc.CASES[case]
    N = spec["N"]
    gold = np.load(os.path.join(GOLDEN, f"gate_{case}.npz"))
    m, mesh = _mesh(N)
    assert int(gold["K"]) == mesh.K and int(gold["N"]) == N
    phys = gc.physics(case)
    q0 = euler.initial_state(gc.initial_primitive(case, mesh.x, phys.rho0, phys.p0, phys.gamma),
                             phys.gamma)
    precision, bar = {"fp32": (dg.DG_FP32, 1e-5), "bf16": (dg.DG_SPLIT_BF16, 1e-3)}[form]
    print(f"gate {case} {form}: K={mesh.K} N={N}", flush=True)
    ctx = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], N, precision=precision,
                           **phys_kwargs(phys))
    perm = node_perm(ctx, mesh.ref)
    qd = torch.tensor((q0 - phys.q0[None, :, None])[:, :, perm], dtype=torch.float32,
                      device="cuda").contiguous()
    res = torch.zeros_like(qd)
    t, _ = dg.dg_run(ctx, qd, res, gc.STEPS, gc.CFL, spec["t0"])
    torch.cuda.synchronize()
    x = qd.double().cpu().numpy()
    q = np.empty_like(x)
    q[:, :, perm] = x
    q += phys.q0[None, :, None]
    dp = norms.pressure(q, phys.gamma) - phys.p0
    dref = gold["dp"].astype(np.float64)
    err = norms.l2(mesh, dp - dref) / norms.l2(mesh, dref)
    t_rel = abs(t / float(gold["t"]) - 1)
    print(f"  p' rel L2 {err:.3e} (bar {bar:g}), |p'|max {np.abs(dref).max():.3e}, "
          f"t {t:.6e} (rel diff {t_rel:.1e})", flush=True)
    dg.dg_destroy(ctx)
    assert t_rel < 1e-6
    assert err < bar
