"""The role-specialized stage kernel (dg_set_kernel(ctx, 1): surface and
contraction wavefronts one tile apart) against the FP64 oracle, with the
bars of the tile-cooperative kernel (test_gpu_parity.py): one right-hand
side within 3e-6 relative L2 and 1e-5 node by node per element group (every
element, the all-interior ones, each boundary tag, the last partial tile),
1e-5 for the pressure perturbation after 100 steps; plus partial tiles down
to one element and blocks with several tiles, determinism, agreement with
the other kernel and the learned-ghost path."""
import numpy as np
import pytest

import paper_1710_03887_amd as dg
from oracle import euler, timestep, norms
from oracle import mlp as omlp
from workloads import (box_kuhn, gaussian_pulse, trumpet_domain, BC_OUTFLOW_CHAR, BC_WALL,
                       BC_INFLOW, BC_PASSTHRU, BC_LEARNED)
from workloads.mlp_init import init_params
from helpers import Pair, rel_l2, assert_nodewise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pulse_state(pair, amp=0.1, width=0.3, center=(0.1, -0.05, 0.02), u=0.0):
    phys = pair.phys
    prim = gaussian_pulse(pair.mesh.x, amp * phys.p0, width, center, phys.rho0, phys.p0,
                          phys.gamma)
    prim[..., 1] += u * np.sin(np.pi * pair.mesh.x[..., 1])
    return euler.initial_state(prim, phys.gamma)


def _wave(pair):
    dg.dg_set_kernel(pair.ctx, 1)
    assert dg.dg_get_kernel(pair.ctx) == 1
    return pair


def _rhs(pair, q, t):
    qd = pair.to_device(q)
    rd = torch.full_like(qd, float("nan"))
    dg.dg_rhs(pair.ctx, qd, rd, t)
    torch.cuda.synchronize()
    return pair.rates_from_device(rd)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_rhs_parity_box(N):
    phys = euler.Physics()
    pair = _wave(Pair(box_kuhn(3, jitter=0.05, seed=N), N, phys))
    q = _pulse_state(pair, u=0.05)
    got, r_or = _rhs(pair, q, 0.0), euler.rhs(pair.mesh, q, 0.0, phys)
    err = rel_l2(pair.mesh, got, r_or)
    print(f"N={N} rhs rel L2 {err:.3e}")
    assert err < 3e-6
    assert_nodewise(got, r_or, pair.bc, 1e-5, f"spec N={N}")


@pytest.mark.parametrize("N", [2, 3, 4])
def test_rhs_parity_all_boundary_kinds_moving(N):
    phys = euler.Physics(u0=(0.05, -0.02, 0.01), amp=0.1 / 1.4, alpha=10.35)
    bc = {"x-": BC_INFLOW, "x+": BC_PASSTHRU, "y-": BC_WALL, "y+": BC_WALL,
          "z-": BC_OUTFLOW_CHAR, "z+": BC_OUTFLOW_CHAR}
    pair = _wave(Pair(box_kuhn((4, 3, 3), jitter=0.05, seed=11, bc=bc), N, phys))
    q = _pulse_state(pair, amp=0.05, width=0.5)
    got, r_or = _rhs(pair, q, 0.13), euler.rhs(pair.mesh, q, 0.13, phys)
    err = rel_l2(pair.mesh, got, r_or)
    print(f"N={N} mixed-boundary rhs rel L2 {err:.3e}")
    assert err < 3e-6
    assert_nodewise(got, r_or, pair.bc, 1e-5, f"spec mixed N={N}")


def test_partial_tiles():
    """K from 6 to 4,500 tets: one partial tile; a few tiles over fewer
    blocks than CUs; several tiles per block (the three-deep pipeline),
    each with a partial last tile."""
    phys = euler.Physics()
    for n in ((1, 1, 1), (2, 1, 1), (3, 2, 1), (5, 3, 2), (15, 10, 5)):
        pair = _wave(Pair(box_kuhn(n, jitter=0.0), 3, phys))
        q = _pulse_state(pair, width=0.8)
        got, r_or = _rhs(pair, q, 0.0), euler.rhs(pair.mesh, q, 0.0, phys)
        err = rel_l2(pair.mesh, got, r_or)
        print(f"{n} hexes ({pair.mesh.K} tets): rhs rel L2 {err:.3e}")
        assert err < 3e-6, (n, err)
        assert_nodewise(got, r_or, pair.bc, 1e-5, f"spec {pair.mesh.K} tets")


def test_run_parity_box_100_steps():
    phys = euler.Physics()
    pair = _wave(Pair(box_kuhn(6, jitter=0.05, seed=0), 2, phys))
    q0 = _pulse_state(pair, amp=0.1, width=0.15, center=(0.0, 0.0, 0.0))
    q_or, t_or, dts = timestep.run(pair.mesh, q0, phys, 100, cfl=0.5)
    qd = pair.to_device(q0)
    res = torch.zeros_like(qd)
    t_gpu, dt_last = dg.dg_run(pair.ctx, qd, res, 100, 0.5, 0.0)
    assert abs(t_gpu / t_or - 1) < 1e-6
    assert abs(dt_last / dts[-1] - 1) < 1e-6
    err = norms.rel_l2_pressure(pair.mesh, pair.from_device(qd), q_or, phys)
    print(f"100 steps p' rel L2 {err:.3e}")
    assert err < 1e-5


def test_trumpet_matches_tile_kernel_and_is_deterministic():
    """Both kernels on a trumpet mesh with every boundary kind of the scene,
    N = 4, 20 steps of dg_run (the time-step rate reduced inside the kernel):
    equal to FP32 rounding; the role-specialized kernel bitwise reproducible
    and its odd-step tail consistent."""
    m = trumpet_domain("box", 6000)
    phys = euler.Physics(amp=0.05 / 1.4, alpha=2 * np.pi * 565.0 / 343.0)
    pair = Pair(m, 4, phys)
    q0 = _pulse_state(pair, amp=0.02, width=0.2, center=(1.0, 0.1, 0.0))
    outs = {}
    for variant in (0, 1, 1):
        dg.dg_set_kernel(pair.ctx, variant)
        qd = pair.to_device(q0)
        res = torch.zeros_like(qd)
        t, _ = dg.dg_run(pair.ctx, qd, res, 20, 0.5, 0.1)
        outs.setdefault(variant, []).append((qd.clone(), t))
    (q_a, t_a), = outs[0]
    (q_b, t_b), (q_c, t_c) = outs[1]
    assert torch.equal(q_b, q_c) and t_b == t_c
    err = norms.rel_l2_pressure(pair.mesh, pair.from_device(q_b), pair.from_device(q_a), phys)
    print(f"role-specialized vs tile kernel after 20 steps: p' rel L2 {err:.3e}")
    assert err < 1e-5 and abs(t_a / t_b - 1) < 1e-6
    qd = pair.to_device(q0)
    res = torch.zeros_like(qd)
    t, _ = dg.dg_run(pair.ctx, qd, res, 7, 0.5, 0.1)
    dg.dg_run(pair.ctx, qd, res, 13, 0.5, t)
    assert torch.equal(qd, q_b)


def test_learned_ghost_path():
    """Learned faces read their ghost traces from the network's buffer."""
    bc = {"x-": BC_LEARNED, "x+": BC_LEARNED, "y-": BC_OUTFLOW_CHAR, "y+": BC_OUTFLOW_CHAR,
          "z-": BC_OUTFLOW_CHAR, "z+": BC_OUTFLOW_CHAR}
    phys = euler.Physics()
    pair = _wave(Pair(box_kuhn(2, jitter=0.05, seed=2, bc=bc), 4, phys))
    prim = gaussian_pulse(pair.mesh.x, 0.05 * phys.p0, 0.4, (0.6, 0.1, 0.0), phys.rho0, phys.p0,
                          phys.gamma)
    prim[..., 1] += 0.01
    q = euler.initial_state(prim, phys.gamma)
    p = init_params(4).astype(np.float32)
    p[128 * 78 + 128 + 128 * 128 + 128:] *= 0.05
    net = dg.dg_mlp_create(p)
    dg.dg_set_learned_bc(pair.ctx, net, 0.0, 1e-4, 1.0, blend=0.6)
    closure = omlp.closure(p.astype(np.float64), phys, 0.0, (2e-4, 0.5), blend=0.6)
    err = rel_l2(pair.mesh, _rhs(pair, q, 0.0), euler.rhs(pair.mesh, q, 0.0, phys, learned=closure))
    print(f"learned rhs rel L2 {err:.3e}")
    assert err < 2e-3


def test_variant_rejected_where_not_supported():
    phys = euler.Physics()
    pair = Pair(box_kuhn(1), 5, phys)
    with pytest.raises(dg.DGError):
        dg.dg_set_kernel(pair.ctx, 1)
    pair = Pair(box_kuhn(1), 3, phys, precision=dg.DG_SPLIT_BF16)
    with pytest.raises(dg.DGError):
        dg.dg_set_kernel(pair.ctx, 1)
