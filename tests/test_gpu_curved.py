"""Curved (isoparametric) elements (dg_set_curved) against the FP64 curved
oracle, on a box whose x = 1 face is bent onto a spherical cap: one
right-hand side (as for straight meshes: FP32 3e-6 relative L2 and 1e-5 node
by node per element group, split-BF16 2e-4 and 1e-3), with an absorbing
layer, with the role-specialized stage kernel, 100 LSERK steps under the
CFL rule (1e-5 for p'), and the error paths."""
import numpy as np
import pytest

import paper_1710_03887_amd as dg
from oracle import euler, timestep, norms, curved
from workloads import gaussian_pulse, BC_OUTFLOW_CHAR, BC_WALL, BC_INFLOW, BC_PASSTHRU
from workloads.curved import capped_box, curved_nodes
from helpers import Pair, rel_l2, rel_l2_rows, assert_nodewise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BC = {"x-": BC_INFLOW, "x+": BC_OUTFLOW_CHAR, "y-": BC_WALL, "y+": BC_PASSTHRU,
      "z-": BC_OUTFLOW_CHAR, "z+": BC_OUTFLOW_CHAR}


def _setup(N, phys, n=(4, 3, 3), precision=dg.DG_FP32, x0=0.0):
    m = capped_box(n, x0=x0, bc=BC)
    pair = Pair(m, N, phys, precision=precision)
    geo = curved.CurvedGeometry(pair.mesh, curved_nodes(m, pair.ref.rst))
    x_lib = curved_nodes(m, dg.dg_reference_operators(pair.ctx)["rst"])
    n_curved = dg.dg_set_curved(pair.ctx, x_lib)
    moved = np.abs(geo.x - pair.mesh.x).max(axis=(1, 2))
    assert n_curved == int(np.sum(moved > 1e-8)) and 0 < n_curved <= pair.mesh.K
    return m, pair, geo, x_lib


@pytest.mark.parametrize("N,moving,variant,precision,layer", [
    (2, False, 0, dg.DG_FP32, False), (3, True, 0, dg.DG_FP32, False),
    (4, False, 0, dg.DG_FP32, False), (4, True, 1, dg.DG_FP32, False),
    (4, False, 0, dg.DG_SPLIT_BF16, False), (5, False, 0, dg.DG_FP32, False),
    (3, False, 0, dg.DG_FP32, True)])
def test_rhs_parity_curved(N, moving, variant, precision, layer):
    phys = euler.Physics(u0=(0.03, 0.0, -0.02) if moving else (0.0, 0.0, 0.0),
                         amp=0.05 / 1.4, alpha=10.35)
    m, pair, geo, _ = _setup(N, phys, precision=precision)
    if variant:
        dg.dg_set_kernel(pair.ctx, variant)
    prim = gaussian_pulse(geo.x, 0.05 * phys.p0, 0.5, (0.6, 0.1, 0.0), phys.rho0, phys.p0,
                          phys.gamma)
    q = euler.initial_state(prim, phys.gamma)
    sig = None
    if layer:
        sig = 3.0 * np.clip(geo.x[..., 0] - 0.3, 0.0, None) ** 2
        sd = torch.tensor(sig[:, pair.perm], dtype=torch.float32, device="cuda").contiguous()
        dg.dg_set_damping(pair.ctx, sd)
    qd = pair.to_device(q)
    rd = torch.full_like(qd, float("nan"))
    dg.dg_rhs(pair.ctx, qd, rd, 0.13)
    torch.cuda.synchronize()
    r_or = curved.rhs(pair.mesh, geo, q, 0.13, phys, sigma=sig)
    got = pair.rates_from_device(rd)
    err = rel_l2(pair.mesh, got, r_or)
    tol = 2e-4 if precision == dg.DG_SPLIT_BF16 else 3e-6
    rows = np.nonzero(np.abs(geo.x - pair.mesh.x).max(axis=(1, 2)) > 1e-8)[0]
    err_c = rel_l2_rows(pair.mesh, rows, got[rows], r_or[rows])
    gap = rel_l2(pair.mesh, euler.rhs(pair.mesh, q, 0.13, phys, sigma=sig), r_or)
    print(f"N={N} moving={moving} variant={variant} precision={precision} layer={layer}: "
          f"rhs rel L2 {err:.3e} (curved rows {err_c:.3e}); straight operator differs by {gap:.2e}")
    assert err < tol and err_c < 5 * tol
    assert gap > 1e-2
    assert_nodewise(got, r_or, pair.bc, 1e-3 if precision == dg.DG_SPLIT_BF16 else 1e-5,
                    f"curved N={N}")


@pytest.mark.parametrize("N,n,x0", [(2, (5, 3, 3), 0.0), (3, (3, 3, 3), -0.999)])
def test_rhs_parity_curved_ragged_and_all(N, n, x0):
    """A curved count that leaves the last block of four wavefronts partly
    empty (162 of 270 elements at N = 2), and every element curved (162 of
    162 at N = 3)."""
    phys = euler.Physics(u0=(0.02, 0.01, 0.0), amp=0.05 / 1.4, alpha=10.35)
    m, pair, geo, _ = _setup(N, phys, n=n, x0=x0)
    q = euler.initial_state(gaussian_pulse(geo.x, 0.05 * phys.p0, 0.5, (0.6, 0.1, 0.0), phys.rho0,
                                           phys.p0, phys.gamma), phys.gamma)
    qd = pair.to_device(q)
    rd = torch.full_like(qd, float("nan"))
    dg.dg_rhs(pair.ctx, qd, rd, 0.07)
    torch.cuda.synchronize()
    got, r_or = pair.rates_from_device(rd), curved.rhs(pair.mesh, geo, q, 0.07, phys)
    err = rel_l2(pair.mesh, got, r_or)
    print(f"N={N} n={n} x0={x0}: rhs rel L2 {err:.3e}")
    assert err < 3e-6
    assert_nodewise(got, r_or, pair.bc, 1e-5, f"curved N={N} n={n}")


def test_stage_matches_rhs_and_clearing():
    """One LSERK stage equals q + b (a res + dt rhs) element by element (the
    stage kernel leaves the curved elements' residual and state to their own
    pass), and clearing the curved set restores the straight-sided operator."""
    phys = euler.Physics()
    m, pair, geo, x_lib = _setup(3, phys)
    prim = gaussian_pulse(geo.x, 0.05 * phys.p0, 0.5, (0.6, 0.1, 0.0), phys.rho0, phys.p0,
                          phys.gamma)
    q = euler.initial_state(prim, phys.gamma)
    qd = pair.to_device(q)
    g = torch.Generator(device="cpu").manual_seed(5)
    res0 = (1e-3 * torch.randn(qd.shape, generator=g, dtype=torch.float32)).cuda()
    res = res0.clone()
    qo = torch.empty_like(qd)
    a, b, dt, t = -0.4178904745, 0.3792103129, 2e-3, 0.05
    dg.dg_stage(pair.ctx, qd, qo, res, a, b, t, dt)
    rd = torch.empty_like(qd)
    dg.dg_rhs(pair.ctx, qd, rd, t)
    torch.cuda.synchronize()
    res_ref = a * res0 + dt * rd
    assert torch.allclose(res, res_ref, rtol=1e-5, atol=1e-9)
    assert torch.allclose(qo, qd + b * res_ref, rtol=1e-6, atol=1e-8)
    assert dg.dg_set_curved(pair.ctx, None) == 0
    dg.dg_rhs(pair.ctx, qd, rd, t)
    torch.cuda.synchronize()
    assert rel_l2(pair.mesh, pair.rates_from_device(rd), euler.rhs(pair.mesh, q, t, phys)) < 2e-5


def test_run_parity_curved_100_steps():
    phys = euler.Physics(amp=0.05 / 1.4, alpha=10.35)
    m, pair, geo, _ = _setup(2, phys, n=(4, 3, 3))
    prim = gaussian_pulse(geo.x, 0.1 * phys.p0, 0.3, (0.5, 0.0, 0.0), phys.rho0, phys.p0,
                          phys.gamma)
    q0 = euler.initial_state(prim, phys.gamma)
    q_or, t_or, dts = timestep.run(pair.mesh, q0, phys, 100, cfl=0.5,
                                   rhs_fn=lambda qq, tt: curved.rhs(pair.mesh, geo, qq, tt, phys))
    qd = pair.to_device(q0)
    res = torch.zeros_like(qd)
    t, _ = dg.dg_run(pair.ctx, qd, res, 100, 0.5, 0.0)
    assert abs(t / t_or - 1) < 1e-6
    err = norms.rel_l2_pressure(pair.mesh, pair.from_device(qd), q_or, phys)
    q_flat, _, _ = timestep.run(pair.mesh, q0, phys, 100, dts=dts)
    gap = norms.rel_l2_pressure(pair.mesh, q_flat, q_or, phys)
    print(f"100 steps, curved cap: p' rel L2 {err:.3e} (straight operator differs by {gap:.2e})")
    assert err < 1e-5 and gap > 1e-3


def test_errors():
    phys = euler.Physics()
    m, pair, geo, x_lib = _setup(2, phys, n=(2, 2, 2))
    with pytest.raises(dg.DGError):
        dg.dg_batch_create([pair.ctx], 4)
    with pytest.raises(dg.DGError):
        dg.dg_set_curved(pair.ctx, x_lib, tol=0.0)
    # a face node moved on one side only: the faces no longer coincide
    mapP = dg.dg_geometry(pair.ctx)["mapP"]
    Fmask = dg.dg_reference_operators(pair.ctx)["Fmask"]
    k, f = [(k, f) for k in range(pair.ctx.K) for f in range(4) if mapP[k, f, 0] >= 0][0]
    bad = x_lib.copy()
    bad[k, Fmask[f, -1]] += 1e-3
    with pytest.raises(dg.DGError):
        dg.dg_set_curved(pair.ctx, bad)
    # an inverted element
    bad = x_lib.copy()
    bad[0] = bad[0][::-1]
    with pytest.raises(dg.DGError):
        dg.dg_set_curved(pair.ctx, bad)
    # after an error the context has no curved set: the straight-sided operator
    q = euler.initial_state(gaussian_pulse(pair.mesh.x, 0.05 * phys.p0, 0.5, (0.2, 0.1, 0.0),
                                           phys.rho0, phys.p0, phys.gamma), phys.gamma)
    qd = pair.to_device(q)
    rd = torch.empty_like(qd)
    dg.dg_rhs(pair.ctx, qd, rd, 0.0)
    torch.cuda.synchronize()
    assert rel_l2(pair.mesh, pair.rates_from_device(rd), euler.rhs(pair.mesh, q, 0.0, phys)) < 2e-5
    quad = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], 2, quadrature=True)
    with pytest.raises(dg.DGError):
        dg.dg_set_curved(quad, curved_nodes(m, dg.dg_reference_operators(quad)["rst"]))
    dg.dg_destroy(quad)


def test_sphere_domain_sampled_parity():
    """The measured workload: the spherical trumpet domain (about 80,000
    tets, N = 4) with its outer side faces laid onto the sphere, in the
    autotuned launch configuration; dg_rhs on sampled curved and straight
    elements against the oracle on their neighbour patch."""
    from workloads import trumpet_domain
    from workloads.curved import sphere_domain_map
    from helpers import face_keys, neighbour_patch, node_perm, phys_kwargs, ref_of
    from oracle.mesh import Mesh
    phys = euler.Physics(amp=0.1 / 1.4, alpha=2 * np.pi * 565.0 / 343.0)
    m = sphere_domain_map(trumpet_domain("sphere", 80_000))
    N = 4
    ctx = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], N, **phys_kwargs(phys))
    x_lib = curved_nodes(m, dg.dg_reference_operators(ctx)["rst"])
    n_curved = dg.dg_set_curved(ctx, x_lib)
    K, Np = ctx.K, ctx.Np
    assert 0.05 * K < n_curved < 0.5 * K
    q0 = torch.zeros((K, 5, Np), dtype=torch.float32, device="cuda")
    dg.dg_autotune(ctx, q0, torch.zeros_like(q0))
    center, width = (0.5, 1.1, 0.4), 0.4
    q_lib = euler.initial_state(gaussian_pulse(x_lib, 0.05 * phys.p0, width, center, phys.rho0,
                                               phys.p0, phys.gamma), phys.gamma)
    qd = torch.tensor(q_lib - phys.q0[None, :, None], dtype=torch.float32, device="cuda")
    rd = torch.empty_like(qd)
    dg.dg_rhs(ctx, qd, rd, 0.02)
    torch.cuda.synchronize()
    got_all = rd.double().cpu().numpy()
    moved = np.abs(x_lib - dg.dg_nodes(ctx)).max(axis=(1, 2)) > 1e-8
    rng = np.random.Generator(np.random.PCG64(11))
    # curved elements where the pulse is, plus straight ones
    xc = x_lib.mean(axis=1)
    near = np.linalg.norm(xc - np.array(center), axis=1) < 2 * width
    sample = np.sort(np.concatenate([rng.choice(np.nonzero(moved & near)[0], 48, replace=False),
                                     rng.choice(np.nonzero(~moved & near)[0], 16, replace=False)]))
    idx, pm = neighbour_patch(m, sample, face_keys(m["EToV"]))
    pm["param"], pm["phi"] = m["param"][idx], m["phi"]
    ref = ref_of(N)
    mesh = Mesh(ref, pm["xyz"], pm["EToV"], pm["bc"])
    geo = curved.CurvedGeometry(mesh, curved_nodes(pm, ref.rst))
    q = euler.initial_state(gaussian_pulse(geo.x, 0.05 * phys.p0, width, center, phys.rho0,
                                           phys.p0, phys.gamma), phys.gamma)
    r_or = curved.rhs(mesh, geo, q, 0.02, phys)
    rows = np.searchsorted(idx, sample)
    perm = node_perm(ctx, ref)
    got = np.empty((len(sample), 5, Np))
    got[:, :, perm] = got_all[sample]
    err = rel_l2_rows(mesh, rows, got, r_or[rows])
    c = np.isin(sample, np.nonzero(moved)[0])
    err_c = rel_l2_rows(mesh, rows[c], got[c], r_or[rows[c]])
    print(f"sphere domain K={K}, {n_curved} curved: sampled rhs rel L2 {err:.3e} "
          f"(curved rows {err_c:.3e})")
    assert err < 2e-5 and err_c < 5e-5
    dg.dg_destroy(ctx)


def test_probe_sample_in_curved_elements():
    """p' sampled by the probe kernel at points inside curved elements (the
    curved map inverted at setup) against the oracle's interpolation of the
    same state at the same reference points."""
    from oracle import probes
    phys = euler.Physics()
    m, pair, geo, _ = _setup(3, phys)
    moved = np.abs(geo.x - pair.mesh.x).max(axis=(1, 2)) > 1e-8
    rng = np.random.default_rng(7)
    rows = rng.choice(np.nonzero(moved)[0], 12, replace=False)
    ref = pair.ref
    lam = rng.dirichlet(np.ones(4), size=len(rows)) * 0.4 + 0.15
    r0 = 2.0 * lam[:, 1:] - 1.0
    pts = np.stack([(probes.weights(ref, r0[i][None]) @ geo.x[k])[0] for i, k in enumerate(rows)])
    q = euler.initial_state(gaussian_pulse(geo.x, 0.05 * phys.p0, 0.5, (0.6, 0.1, 0.0), phys.rho0,
                                           phys.p0, phys.gamma), phys.gamma)
    e_or, rst = curved.locate(pair.mesh, geo, pts, moved)
    p_or = probes.sample(pair.mesh, q, e_or, probes.weights(ref, rst), phys)
    dg.dg_probe_setup(pair.ctx, pts)
    out = torch.empty(len(pts), dtype=torch.float32, device="cuda")
    dg.dg_probe_sample(pair.ctx, pair.to_device(q), out)
    torch.cuda.synchronize()
    got = out.double().cpu().numpy()
    err = np.abs(got - p_or).max() / np.abs(p_or).max()
    print(f"curved probes: max rel difference {err:.2e}")
    assert err < 1e-5
