"""GPU tests of batched ensembles: several geometries x 16 inflow-pulse
amplitudes advanced by one persistent stage launch per RK stage.

Amplitudes are the ensemble's, log-spaced p0 10^(-3 + 2 i / 15), i = 0..15
(0.1 % to 10 %).  Each member is an independent solve, so
  * against the FP64 oracle it meets the same bar as a single solve
    (pressure-perturbation relative L2 1e-5 after 100 steps, end time within
    1e-6 relative -- the batch takes its own CFL steps per member), checked
    for the smallest amplitude on the box, the median on the sphere and the
    largest on the half domain against the oracle's results stored by
    tests/golden/make_gates.py;
  * against the single-solve library path (same FP32 arithmetic, different
    accumulation order) it meets the same 1e-5 bar;
  * it is bitwise independent of the other members, of the other
    geometries in the batch, of the number of active members and of the
    launch shape (MFMA columns never mix, reductions are maxima).
"""
import os

import numpy as np
import pytest

import paper_1710_03887_amd as dg
import gate_cases as gc
from oracle import euler, norms
from workloads import trumpet_domain
from helpers import Pair

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N = 3
ALPHA = 2 * np.pi * 565.0 / 343.0
P0 = 1.0 / 1.4
T_START = gc.ENSEMBLE_T0          # inside the raised-cosine pulse (period 343/565)
AMPS = P0 * gc.ENSEMBLE_AMPS
KINDS = ("box", "sphere", "half")
GEOMS = [trumpet_domain(kind, 1500) for kind in KINDS]
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _phys(amp):
    return euler.Physics(amp=amp, alpha=ALPHA)


def _start_state(pair):
    """Quiet fluid with a weak Gaussian bump near the bore, so that volume,
    interior-face and every boundary term are active from the first stage."""
    phys = pair.phys
    prim = gc.initial_primitive("c4_box_m0", pair.mesh.x, phys.rho0, phys.p0, phys.gamma)
    return euler.initial_state(prim, phys.gamma)


def _to_batch(pair, q_oracle):
    x = pair.to_device(q_oracle)                       # [K,5,Np]
    return x[..., None].expand(*x.shape, 16).contiguous().clone()


def _member(pair, qb, e):
    return pair.from_device(qb[..., e].contiguous())


@pytest.fixture(scope="module")
def setup():
    pairs = [Pair(m, N, _phys(AMPS[0])) for m in GEOMS]
    starts = [_start_state(p) for p in pairs]
    return pairs, starts


def _run_batch(pairs, starts, nsteps, amps=None, members=16, launch=None, idx=None):
    idx = list(range(len(pairs))) if idx is None else idx
    b = dg.dg_batch_create([pairs[i].ctx for i in idx], members)
    if launch:
        dg.dg_batch_set_launch(b, *launch)
    q = [_to_batch(pairs[i], starts[i]) for i in idx]
    res = [torch.zeros_like(x) for x in q]
    amps = np.broadcast_to(AMPS if amps is None else amps, (len(idx), 16))
    t = dg.dg_batch_run(b, q, res, amps, nsteps, 0.5, np.full((len(idx), 16), T_START))
    torch.cuda.synchronize()
    return q, t, b


@pytest.mark.timeout(300)
def test_batch_matches_oracle_100_steps(setup):
    pairs, starts = setup
    q, t, _ = _run_batch(pairs, starts, gc.STEPS)
    for kind, e in gc.ENSEMBLE_SAMPLES:
        g = KINDS.index(kind)
        gold = np.load(os.path.join(GOLDEN, f"gate_c4_{kind}_m{e}.npz"))
        pair = pairs[g]
        assert int(gold["K"]) == pair.mesh.K
        t_or = float(gold["t"])
        assert abs((t[g, e] - T_START) / (t_or - T_START) - 1) < 1e-6
        q_gpu = _member(pair, q[g], e)
        dp = norms.pressure(q_gpu, pair.phys.gamma) - pair.phys.p0
        dref = gold["dp"].astype(np.float64)
        err = norms.l2(pair.mesh, dp - dref) / norms.l2(pair.mesh, dref)
        print(f"{kind} member {e} (amplitude {AMPS[e] / P0:.4%} p0): 100-step p' rel L2 {err:.3e}")
        assert err < 1e-5


def test_batch_matches_single_solve(setup):
    pairs, starts = setup
    q, t, _ = _run_batch(pairs, starts, 12)
    for g in range(3):
        for e in (0, 9):
            m, G = pairs[g], GEOMS[g]
            ctx = dg.dg_mesh_setup(G["xyz"], G["EToV"], G["bc"], N, p0=P0, inflow_amp=AMPS[e],
                                   inflow_alpha=ALPHA)
            qd = m.to_device(starts[g])
            res = torch.zeros_like(qd)
            t1, _ = dg.dg_run(ctx, qd, res, 12, 0.5, T_START)
            assert abs((t[g, e] - T_START) / (t1 - T_START) - 1) < 1e-6
            err = norms.rel_l2_pressure(m.mesh, _member(m, q[g], e), m.from_device(qd), m.phys)
            assert err < 1e-5, (g, e, err)


def test_member_permutation_is_bitwise(setup):
    pairs, starts = setup
    perm = np.random.default_rng(4).permutation(16)
    q1, t1, _ = _run_batch(pairs, starts, 5)
    q2, t2, _ = _run_batch(pairs, starts, 5, amps=AMPS[perm])
    for g in range(3):
        assert torch.equal(q2[g], q1[g][..., torch.as_tensor(perm, device=q1[g].device)])
        assert np.array_equal(t2[g], t1[g][perm])


def test_geometry_subset_active_members_and_launch_shape_are_bitwise(setup):
    pairs, starts = setup
    q_all, t_all, _ = _run_batch(pairs, starts, 5)
    q_one, t_one, _ = _run_batch(pairs, starts, 5, idx=[1])
    assert torch.equal(q_one[0], q_all[1]) and np.array_equal(t_one[0], t_all[1])
    q5, t5, _ = _run_batch(pairs, starts, 5, members=5)
    for g in range(3):
        assert torch.equal(q5[g][..., :5], q_all[g][..., :5])
        assert np.array_equal(t5[g][:5], t_all[g][:5])
    for launch in ((1, 1), (0, 8), (2, 2)):
        ql, tl, _ = _run_batch(pairs, starts, 5, launch=launch)
        for g in range(3):
            assert torch.equal(ql[g], q_all[g]), launch
            assert np.array_equal(tl[g], t_all[g])


def test_batch_odd_steps_and_restart(setup):
    pairs, starts = setup
    q7, t7, _ = _run_batch(pairs, starts, 7)
    b = dg.dg_batch_create([p.ctx for p in pairs])
    q = [_to_batch(p, s) for p, s in zip(pairs, starts)]
    res = [torch.zeros_like(x) for x in q]
    t = dg.dg_batch_run(b, q, res, np.broadcast_to(AMPS, (3, 16)), 3, 0.5,
                        np.full((3, 16), T_START))
    t = dg.dg_batch_run(b, q, res, np.broadcast_to(AMPS, (3, 16)), 4, 0.5, t)
    torch.cuda.synchronize()
    for g in range(3):
        assert torch.equal(q[g], q7[g])
    assert np.array_equal(t, t7)


def test_batch_nonphysical_member_is_reported(setup):
    pairs, starts = setup
    b = dg.dg_batch_create([p.ctx for p in pairs])
    q = [_to_batch(p, s) for p, s in zip(pairs, starts)]
    q[2][7, 0, :, 3] = -2.0                  # negative density, geometry 2 member 3
    res = [torch.zeros_like(x) for x in q]
    with pytest.raises(dg.DGError) as e:
        dg.dg_batch_run(b, q, res, np.broadcast_to(AMPS, (3, 16)), 2, 0.5,
                        np.full((3, 16), T_START))
    assert e.value.code == dg.DG_ENONPHYS
    fb = dg.dg_batch_first_bad(b)
    expect = np.full((3, 16), -1)
    expect[2, 3] = 0
    assert np.array_equal(fb, expect)


def test_batch_rejects_mismatched_contexts(setup):
    pairs, _ = setup
    m = GEOMS[0]
    other = dg.dg_mesh_setup(m["xyz"], m["EToV"], m["bc"], 2)
    with pytest.raises(dg.DGError):
        dg.dg_batch_create([pairs[0].ctx, other])
    with pytest.raises(dg.DGError):
        dg.dg_batch_create([pairs[0].ctx], members=17)


def test_autotuners_keep_state_and_use_cache(setup, tmp_path):
    pairs, starts = setup
    cache = str(tmp_path / "tune.txt")
    b = dg.dg_batch_create([p.ctx for p in pairs])
    q = [_to_batch(p, s) for p, s in zip(pairs, starts)]
    q_copy = [x.clone() for x in q]
    res = [torch.zeros_like(x) for x in q]
    shape = dg.dg_batch_autotune(b, q, res, cache)
    assert shape[1] in (1, 2, 4, 8) and shape[0] >= 1
    assert all(torch.equal(a, c) for a, c in zip(q, q_copy))
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("batch/N3/m16/K")
    assert dg.dg_batch_autotune(b, q, res, cache) == shape      # from the cache
    assert len(open(cache).read().splitlines()) == 1
    # the tuned batch gives the untuned batch's results
    t = dg.dg_batch_run(b, q, res, np.broadcast_to(AMPS, (3, 16)), 5, 0.5,
                        np.full((3, 16), T_START))
    torch.cuda.synchronize()
    q_ref, t_ref, _ = _run_batch(pairs, starts, 5)
    assert all(torch.equal(a, c) for a, c in zip(q, q_ref)) and np.array_equal(t, t_ref)

    pair = pairs[0]
    qd = pair.to_device(starts[0])
    before = qd.clone()
    r = torch.zeros_like(qd)
    bpc = dg.dg_autotune(pair.ctx, qd, r, cache)
    assert bpc >= 1 and torch.equal(qd, before)
    assert dg.dg_autotune(pair.ctx, qd, r, cache) == bpc
    assert len(open(cache).read().splitlines()) == 2


@pytest.mark.timeout(600)
def test_full_size_members_match_single_solves():
    """The ensemble at its full size, in the launch shape the benchmark uses
    (the autotuner's): the box, sphere and half domains at 49,536, 80,370
    and 31,980 tets, N = 3, 16 members each, one launch per stage.  After 3
    steps the members at 0.1 %, 1.2 % and 10 % p0 of every geometry match
    single solves of the same geometry and amplitude (the library path the
    full-size and 100-step tests pin to the oracle) within the same 1e-5
    bar, with the same end time."""
    sizes = (("box", 50_000, 49_536), ("sphere", 80_000, 80_370), ("half", 30_000, 31_980))
    geoms = [trumpet_domain(kind, n) for kind, n, _ in sizes]
    assert [len(g["EToV"]) for g in geoms] == [k for _, _, k in sizes]
    pairs = [Pair(m, N, _phys(AMPS[0])) for m in geoms]
    starts = [_start_state(p) for p in pairs]
    b = dg.dg_batch_create([p.ctx for p in pairs], 16)
    q = [_to_batch(p, s) for p, s in zip(pairs, starts)]
    res = [torch.zeros_like(x) for x in q]
    bpc, waves = dg.dg_batch_autotune(b, q, res, None)
    print(f"launch shape: {bpc} blocks per CU, {waves} wavefronts per block")
    amps = np.broadcast_to(AMPS, (3, 16))
    t = dg.dg_batch_run(b, q, res, amps, 3, 0.5, np.full((3, 16), T_START))
    torch.cuda.synchronize()
    for g, G in enumerate(geoms):
        for e in (0, 8, 15):
            ctx = dg.dg_mesh_setup(G["xyz"], G["EToV"], G["bc"], N, p0=P0, inflow_amp=AMPS[e],
                                   inflow_alpha=ALPHA)
            qd = pairs[g].to_device(starts[g])
            r1 = torch.zeros_like(qd)
            t1, _ = dg.dg_run(ctx, qd, r1, 3, 0.5, T_START)
            assert abs((t[g, e] - T_START) / (t1 - T_START) - 1) < 1e-6
            err = norms.rel_l2_pressure(pairs[g].mesh, _member(pairs[g], q[g], e),
                                        pairs[g].from_device(qd), pairs[g].phys)
            print(f"{KINDS[g]} member {e} ({AMPS[e] / P0:.3%} p0): rel L2 {err:.2e}")
            assert err < 1e-5, (g, e, err)
