"""GPU parity of the split-BF16 form against the FP64 oracle.

The volume contraction runs as hi*hi + hi*lo + lo*hi BF16 products with
FP32 accumulation.  Writing x = hi + lo + d with |d| <= 2^-16 |x| (lo is
itself rounded to 8 significant bits) and dropping lo*lo, each product
D_ij F_j is off by at most ~3 * 2^-16 |D_ij F_j|; summed over the Np x 3Np
contraction with the cancellation a derivative has (|sum D F| is ~h^-1 |F|
while sum |D| |F| is ~h^-1 (N+1)^2 |F|), one right-hand side is within
~3 * 2^-16 (N+1)^2 ~ 1e-3 relative at N = 4 in the worst case of aligned
rounding.  The rounding errors are not aligned: 1e-5 relative L2 is observed
(N = 1..5 and the 1.17M-tet N = 5 mesh), so one evaluation is held to 2e-4
relative L2 and, node by node (per variable, per element group: all,
all-interior, each boundary tag, the last partial tile; relative to the
variable's largest value), to 1e-3; 100 steps to the method's 1e-3 relative
L2 of p'.
"""
import numpy as np
import pytest

import paper_1710_03887_amd as dg
from oracle import euler, timestep, norms
from workloads import box_kuhn, gaussian_pulse
from helpers import Pair, rel_l2, assert_nodewise

BF16_L2_BAR = 2e-4
BF16_NODE_BAR = 1e-3

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _state(pair, amp, width=0.3, center=(0.1, -0.05, 0.02)):
    phys = pair.phys
    prim = gaussian_pulse(pair.mesh.x, amp * phys.p0, width, center, phys.rho0, phys.p0,
                          phys.gamma)
    return euler.initial_state(prim, phys.gamma)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_rhs_parity_bf16(N):
    phys = euler.Physics()
    pair = Pair(box_kuhn(3, jitter=0.05, seed=N), N, phys, precision=dg.DG_SPLIT_BF16)
    q = _state(pair, 0.1)
    r_or = euler.rhs(pair.mesh, q, 0.0, phys)
    qd = pair.to_device(q)
    rd = torch.empty_like(qd)
    dg.dg_rhs(pair.ctx, qd, rd, 0.0)
    torch.cuda.synchronize()
    r_gpu = pair.rates_from_device(rd)
    err = rel_l2(pair.mesh, r_gpu, r_or)
    print(f"N={N} split-BF16 rhs rel L2 {err:.3e}")
    assert err < BF16_L2_BAR
    assert_nodewise(r_gpu, r_or, pair.bc, BF16_NODE_BAR, f"N={N} bf16")


@pytest.mark.parametrize("amp", [0.005, 0.02, 0.1])
def test_run_parity_bf16_amplitudes(amp):
    """100 steps at 0.5 %, 2 % and 10 % of p0 (N = 3, jittered box,
    characteristic outflow): p' within 1e-3 relative L2 of the oracle."""
    phys = euler.Physics()
    pair = Pair(box_kuhn(4, jitter=0.05, seed=7), 3, phys, precision=dg.DG_SPLIT_BF16)
    q0 = _state(pair, amp, width=0.25, center=(0.0, 0.0, 0.0))
    q_or, t_or, dts = timestep.run(pair.mesh, q0, phys, 100, cfl=0.5)
    qd = pair.to_device(q0)
    res = torch.zeros_like(qd)
    t_gpu, _ = dg.dg_run(pair.ctx, qd, res, 100, 0.5, 0.0)
    assert abs(t_gpu / t_or - 1) < 1e-6
    err = norms.rel_l2_pressure(pair.mesh, pair.from_device(qd), q_or, phys)
    print(f"amp {amp}: split-BF16 100-step p' rel L2 {err:.3e}")
    assert err < 1e-3
