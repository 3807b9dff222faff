"""Writes the expected results of the 100-step accuracy gates with the FP64
oracle alone (nothing here calls the library):

    python tests/golden/make_gates.py [case ...]     # default: every case

For each case of tests/gate_cases.py it runs the oracle's LSERK4 for 100
steps at CFL 0.5 from the case's initial state and stores, in
tests/golden/gate_<case>.npz, the pressure perturbation p - p0 at every node
(oracle node order, FP32: its rounding, 6e-8 relative, is far below the
1e-5 bar), the end time, the time steps and the mesh size.  One process per
case, each on one BLAS thread.
"""
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))


def run_case(case):
    from threadpoolctl import threadpool_limits
    import gate_cases as gc
    from oracle import euler, timestep, norms
    from oracle.mesh import Mesh
    from oracle.operators import RefElement
    spec = gc.CASES[case]
    m = gc.mesh(case)
    phys = gc.physics(case)
    mesh = Mesh(RefElement(spec["N"]), m["xyz"], m["EToV"], m["bc"])
    q0 = euler.initial_state(gc.initial_primitive(case, mesh.x, phys.rho0, phys.p0, phys.gamma),
                             phys.gamma)
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        q, t, dts = timestep.run(mesh, q0, phys, gc.STEPS, cfl=gc.CFL, t0=spec["t0"])
    dp = norms.pressure(q, phys.gamma) - phys.p0
    np.savez_compressed(os.path.join(HERE, f"gate_{case}.npz"), dp=dp.astype(np.float32),
                        t=np.float64(t), dts=np.array(dts), K=np.int64(mesh.K),
                        N=np.int64(spec["N"]))
    return case, mesh.K, t, time.perf_counter() - t0


if __name__ == "__main__":
    import gate_cases as gc
    cases = sys.argv[1:] or list(gc.CASES)
    with mp.get_context("spawn").Pool(len(cases)) as pool:
        for case, K, t, secs in pool.imap_unordered(run_case, cases):
            print(json.dumps({"case": case, "K": K, "t_end": t, "oracle_seconds": round(secs, 1)}),
                  flush=True)
