"""The precision workload at full size: the trumpet in the box refined to
1,165,248 tetrahedra at N = 5 (Np = 56), FP32 and split-BF16 forms, each in
the launch configuration its autotuner picks.  One right-hand side of the
whole mesh on the GPU; the FP64 oracle evaluates the same right-hand side
element by element on a sample (2,000 random elements plus 200 touching each
boundary kind), on the patch made of the sample and its face neighbours, so
every sampled element sees exactly its full-mesh neighbourhood.  Bars as for
the small cases: FP32 3e-6 relative L2 over all variables of the sampled
elements and 1e-5 node by node, split-BF16 2e-4 and 1e-3 (see
test_gpu_parity.py and test_gpu_bf16.py).

The 100-step comparison at 0.5 %, 2 % and 10 % p0 on a 19,530-tet
subsample is in test_gpu_gates.py."""
import numpy as np
import pytest

import paper_1710_03887_amd as dg
from oracle import euler
from oracle.mesh import Mesh
from oracle.nodes import barycentric
from workloads import trumpet_domain, gaussian_pulse, BC_OUTFLOW_CHAR, BC_WALL, BC_INFLOW
from helpers import (ref_of, node_perm, phys_kwargs, face_keys, neighbour_patch, oriented_nodes,
                     rel_l2_rows, assert_nodewise)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ALPHA = 2 * np.pi * 565.0 / 343.0


def _state(x, phys):
    prim = gaussian_pulse(x, 0.05 * phys.p0, 0.2, (0.85, 0.05, 0.0), phys.rho0, phys.p0,
                          phys.gamma)
    prim[..., 2] += 0.02 * np.exp(-((x[..., 0] - 1.2) ** 2) / 0.3)
    return euler.initial_state(prim, phys.gamma)


@pytest.mark.timeout(600)
def test_rhs_parity_full_size_n5():
    N = 5
    m = trumpet_domain("box", 1_200_000)
    K = m["EToV"].shape[0]
    assert K == 1_165_248
    phys = euler.Physics(amp=0.1 / 1.4, alpha=ALPHA)
    ref = ref_of(N)
    t_peak = np.pi / ALPHA

    rng = np.random.default_rng(5)
    sample = [rng.choice(K, 2000, replace=False)]
    for tag in (BC_WALL, BC_INFLOW, BC_OUTFLOW_CHAR):
        cand = np.nonzero((m["bc"] == tag).any(axis=1))[0]
        sample.append(rng.choice(cand, min(200, cand.size), replace=False))
    sample = np.unique(np.concatenate(sample))
    keys = face_keys(m["EToV"])
    idx, pm = neighbour_patch(m, sample, keys)
    pmesh = Mesh(ref, pm["xyz"], pm["EToV"], pm["bc"])
    rows = np.searchsorted(idx, sample)
    r_or = euler.rhs(pmesh, _state(pmesh.x, phys), t_peak, phys)[rows]

    ctxs = [(dg.DG_FP32, 3e-6, 1e-5), (dg.DG_SPLIT_BF16, 2e-4, 1e-3)]
    lam = barycentric(ref.rst)
    qd = None
    for precision, tol, node_tol in ctxs:
        ctx = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], N, precision=precision,
                               **phys_kwargs(phys))
        perm = node_perm(ctx, ref)
        if qd is None:
            qd = torch.empty((K, 5, ref.Np), dtype=torch.float32, device="cuda")
            for k0 in range(0, K, 100_000):
                k1 = min(K, k0 + 100_000)
                q = _state(oriented_nodes(m["xyz"][k0:k1], lam), phys)
                qp = (q - phys.q0[None, :, None])[:, :, perm]
                qd[k0:k1] = torch.from_numpy(qp.astype(np.float32)).cuda()
        res = torch.zeros_like(qd)
        dg.dg_autotune(ctx, qd, res)
        rd = torch.empty_like(qd)
        dg.dg_rhs(ctx, qd, rd, t_peak)
        torch.cuda.synchronize()
        x = rd[torch.from_numpy(sample).cuda()].double().cpu().numpy()
        r_gpu = np.empty_like(x)
        r_gpu[:, :, perm] = x
        err = rel_l2_rows(pmesh, rows, r_gpu, r_or)
        print(f"precision {precision}: rhs rel L2 {err:.3e} over {sample.size} sampled of {K} "
              f"elements (patch {idx.size}), kernel variant {dg.dg_get_kernel(ctx)}", flush=True)
        assert err < tol
        assert_nodewise(r_gpu, r_or, m["bc"][sample], node_tol, f"N=5 precision {precision}")
        dg.dg_destroy(ctx)
