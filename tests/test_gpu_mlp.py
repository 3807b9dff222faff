"""GPU tests of the learned boundary closure against the FP64 oracle
(oracle/mlp.py): FP32 forward and gradients, one Adam step, BF16 inference,
trace sampling, the learned ghost inside the solver, determinism and a
training run that learns.

Tolerances: FP32 products of length <= 128 with O(1) weights carry relative
errors of a few 1e-7, so the FP32 forward is held to 1e-5 and the gradient
(whose small components are sums of cancelling terms) to 1e-4 of its largest
component.  BF16 rounds weights and activations to 8 significant bits
(relative 2^-9 = 2e-3 each); over three layers of length 78-128 sums with
random signs the output error is ~1e-2 of the output scale, the bar is 3e-2.
"""
import numpy as np
import pytest

import paper_1710_03887_amd as dg
from oracle import mlp as omlp
from oracle import euler
from workloads.mlp_init import init_params
from workloads import box_kuhn, gaussian_pulse, BC_LEARNED, BC_OUTFLOW_CHAR
from helpers import Pair, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _data(B, seed=0, scale=0.5):
    rng = np.random.default_rng(seed)
    X = rng.normal(scale=scale, size=(B, 78))
    n = rng.normal(size=(B, 3))
    X[:, 75:] = n / np.linalg.norm(n, axis=1, keepdims=True)
    Y = rng.normal(scale=scale, size=(B, 75))
    return X, Y


def _dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float32), device="cuda").contiguous()


def _params(seed=0):
    """He-uniform start, then the FP32 values both sides use."""
    return init_params(seed).astype(np.float32)


def test_forward_fp32_and_bf16_match_oracle():
    p = _params(1)
    X, _ = _data(1000, 1)
    Xf = X.astype(np.float32).astype(np.float64)
    Y_or, _ = omlp.forward(p.astype(np.float64), Xf)
    m = dg.dg_mlp_create(p)
    Xd = _dev(X)
    for bf16, tol in ((False, 1e-5), (True, 3e-2)):
        Yd = torch.empty((1000, 75), dtype=torch.float32, device="cuda")
        dg.dg_mlp_infer(m, Xd, Yd, bf16=bf16)
        torch.cuda.synchronize()
        err = np.abs(Yd.cpu().numpy() - Y_or).max() / np.abs(Y_or).max()
        print(f"bf16={bf16}: max rel err {err:.2e}")
        assert err < tol
    # ragged row counts (tiles of 16 and 64 rows)
    for B in (1, 15, 17, 63, 65):
        Yd = torch.empty((B, 75), dtype=torch.float32, device="cuda")
        dg.dg_mlp_infer(m, Xd[:B].contiguous(), Yd, bf16=True)
        torch.cuda.synchronize()
        assert np.abs(Yd.cpu().numpy() - Y_or[:B]).max() / np.abs(Y_or).max() < 3e-2


@pytest.mark.parametrize("rows", [777, 4100])
def test_gradient_matches_oracle(rows):
    """Loss and gradient against the FP64 oracle; 777 rows split the
    weight-gradient products into two chunks (the last one ragged), 4,100
    rows into the most chunks (eight)."""
    p = _params(2)
    X, Y = _data(rows, 2)
    Xf, Yf = X.astype(np.float32).astype(np.float64), Y.astype(np.float32).astype(np.float64)
    L_or, g_or = omlp.grad(p.astype(np.float64), Xf, Yf)
    m = dg.dg_mlp_create(p)
    L, g = dg.dg_mlp_grad(m, _dev(X), _dev(Y))
    g = g.cpu().numpy().astype(np.float64)
    assert abs(L - L_or) / L_or < 1e-5
    err = np.abs(g - g_or).max() / np.abs(g_or).max()
    print(f"gradient max rel err {err:.2e}")
    assert err < 1e-4
    # deterministic
    _, g2 = dg.dg_mlp_grad(m, _dev(X), _dev(Y))
    assert np.array_equal(g2.cpu().numpy().astype(np.float64), g)


def test_adam_step_matches_oracle():
    p = _params(3)
    X, Y = _data(512, 3)
    Xf, Yf = X.astype(np.float32).astype(np.float64), Y.astype(np.float32).astype(np.float64)
    opt = omlp.Adam(p.size)
    pp = p.astype(np.float64)
    for _ in range(3):
        _, g = omlp.grad(pp, Xf, Yf)
        pp = opt.step(pp, g, 1e-3)
    m = dg.dg_mlp_create(p)
    for _ in range(3):
        dg.dg_mlp_train_step(m, _dev(X), _dev(Y), 1e-3)
    q = dg.dg_mlp_get_params(m).astype(np.float64)
    # Adam moves each parameter by about lr per step; compare the moves
    err = np.abs((q - p) - (pp - p)).max()
    print(f"3 Adam steps: max |move difference| {err:.2e} (moves ~3e-3)")
    assert err < 3e-5


def test_training_learns_and_is_deterministic():
    """Fit a fixed linear map of random inputs: the loss must fall by 10x,
    and two runs with the same minibatch sequence are bitwise equal."""
    rng = np.random.default_rng(5)
    B = 8192
    X, _ = _data(B, 5, scale=0.3)
    # target: a fixed linear map of the inputs (learnable exactly)
    A = rng.normal(scale=0.1, size=(78, 75))
    Y = X @ A
    Xd, Yd = _dev(X), _dev(Y)
    out = []
    for _ in range(2):
        m = dg.dg_mlp_create(_params(0))
        gen = np.random.default_rng(7)
        first = last = None
        for it in range(1000):
            rows = torch.tensor(gen.integers(0, B, 512), dtype=torch.int64, device="cuda")
            L = dg.dg_mlp_train_step(m, Xd, Yd, 1e-3, rows=rows, want_loss=it in (0, 999))
            if it == 0:
                first = L
            if it == 999:
                last = L
        out.append(dg.dg_mlp_get_params(m))
        print(f"loss {first:.3e} -> {last:.3e}")
        assert last < first / 10
    assert np.array_equal(out[0], out[1])


def _learned_pair(seed=0):
    """N = 4 box with two opposite faces learned, a pulse crossing them."""
    bc = {"x-": BC_LEARNED, "x+": BC_LEARNED, "y-": BC_OUTFLOW_CHAR, "y+": BC_OUTFLOW_CHAR,
          "z-": BC_OUTFLOW_CHAR, "z+": BC_OUTFLOW_CHAR}
    m = box_kuhn(2, jitter=0.05, seed=seed, bc=bc)
    phys = euler.Physics()
    pair = Pair(m, 4, phys)
    prim = gaussian_pulse(pair.mesh.x, 0.05 * phys.p0, 0.4, (0.6, 0.1, 0.0), phys.rho0, phys.p0,
                          phys.gamma)
    prim[..., 1] += 0.01
    return pair, euler.initial_state(prim, phys.gamma)


@pytest.mark.parametrize("norm", [0.1 / 1.4, 0.0])
def test_sample_traces_match_oracle(norm):
    """Every face of the mesh: X = characteristic ghost of the interior
    trace / scale and the normal; Y = exterior trace / scale: the
    neighbour's trace on interior faces, the ghost of the tag on boundary
    faces (learned faces without a network: the characteristic ghost, so
    Y equals X's trace part there); scale = norm, or the largest |q'| of
    each face's characteristic ghost when norm = 0."""
    pair, q = _learned_pair(1)
    phys = pair.phys
    K = pair.mesh.K
    faces = np.arange(4 * K, dtype=np.int64)
    X = torch.empty((4 * K, 78), dtype=torch.float32, device="cuda")
    Y = torch.empty((4 * K, 75), dtype=torch.float32, device="cuda")
    dg.dg_sample_traces(pair.ctx, pair.to_device(q), torch.tensor(faces, device="cuda"), norm, X, Y)
    torch.cuda.synchronize()
    char = lambda qm, n: euler.ghost_state(euler.OUTFLOW_CHAR, qm, n, phys, 0.0)  # noqa: E731
    qm, qp, nrm = euler.face_traces(pair.mesh, q, 0.0, phys, learned=char)   # [K, 4, Nfp, 5]
    qc = char(qm, nrm)                           # the network's input: characteristic ghost
    dc = np.transpose(qc - phys.q0, (0, 1, 3, 2)).reshape(4 * K, -1)
    sc = omlp.face_scale(dc, norm)
    dc = dc / sc[:, None]
    dp = np.transpose(qp - phys.q0, (0, 1, 3, 2)).reshape(4 * K, -1) / sc[:, None]
    Xo = np.concatenate([dc, pair.mesh.normals.reshape(4 * K, 3)], axis=1)
    assert np.abs(X.cpu().numpy() - Xo).max() < 1e-5 * np.abs(Xo).max()
    assert np.abs(Y.cpu().numpy() - dp).max() < 1e-4 * np.abs(dp).max()
    lrn = pair.mesh.bc.ravel() == BC_LEARNED
    assert np.abs(dp[lrn] - dc[lrn]).max() < 1e-12
    # the learned-face list is exactly the faces tagged learned
    lf = dg.dg_learned_faces(pair.ctx)
    tagged = np.nonzero(pair.mesh.bc.ravel() == BC_LEARNED)[0]
    assert np.array_equal(np.sort(lf), tagged)


def _closure_setup(pair, window, norm=0.1 / 1.4, blend=1.0):
    p = _params(4)
    # damp the output layer so the network's ghost stays near the ambient state
    o3 = 128 * 78 + 128 + 128 * 128 + 128
    p[o3:] *= 0.05
    m = dg.dg_mlp_create(p)
    dg.dg_set_learned_bc(pair.ctx, m, norm, *window, blend=blend)
    return p, m, norm


@pytest.mark.parametrize("norm,blend", [(0.1 / 1.4, 1.0), (0.0, 1.0), (0.0, 0.6)])
def test_learned_ghost_rhs_matches_oracle(norm, blend):
    pair, q = _learned_pair(2)
    phys = pair.phys
    window = (1e-4, 1.0)            # every face with a pulse on it uses the network
    p, m, norm = _closure_setup(pair, window, norm, blend)
    qd = pair.to_device(q)
    rd = torch.empty_like(qd)
    dg.dg_rhs(pair.ctx, qd, rd, 0.0)
    torch.cuda.synchronize()
    closure = omlp.closure(p.astype(np.float64), phys, norm, (2e-4, 0.5), blend=blend)
    r_or = euler.rhs(pair.mesh, q, 0.0, phys, learned=closure)
    r_char = euler.rhs(pair.mesh, q, 0.0, phys,
                       learned=lambda qm, n: euler.ghost_state(euler.OUTFLOW_CHAR, qm, n, phys, 0.0))
    err = rel_l2(pair.mesh, pair.rates_from_device(rd), r_or)
    sep = rel_l2(pair.mesh, r_char, r_or)
    print(f"learned rhs rel L2 vs oracle {err:.2e}; learned vs char {sep:.2e}")
    assert sep > 10 * err          # the network path is really taken
    assert err < 2e-3              # BF16 network inside an FP32 rhs


def test_learned_ghost_window_falls_back_to_characteristic():
    pair, q = _learned_pair(3)
    phys = pair.phys
    _closure_setup(pair, (10.0, 20.0))   # no face reaches the window
    qd = pair.to_device(q)
    rd = torch.empty_like(qd)
    dg.dg_rhs(pair.ctx, qd, rd, 0.0)
    torch.cuda.synchronize()
    r_char = euler.rhs(pair.mesh, q, 0.0, phys,
                       learned=lambda qm, n: euler.ghost_state(euler.OUTFLOW_CHAR, qm, n, phys, 0.0))
    assert rel_l2(pair.mesh, pair.rates_from_device(rd), r_char) < 2e-5
    # detaching gives the in-kernel characteristic ghost
    dg.dg_set_learned_bc(pair.ctx, None, 1.0, 0.0, 0.0)
    rd2 = torch.empty_like(qd)
    dg.dg_rhs(pair.ctx, qd, rd2, 0.0)
    torch.cuda.synchronize()
    assert rel_l2(pair.mesh, pair.rates_from_device(rd2), r_char) < 2e-5


def test_learned_run_graph_uses_current_weights():
    """dg_run replays a captured graph; weight updates made between runs
    must reach it (bf16 weights repacked before the replay)."""
    pair, q = _learned_pair(4)
    p, m, norm = _closure_setup(pair, (1e-4, 1.0))
    outs = []
    for scale in (1.0, 0.5, 1.0):
        pp = p.copy()
        pp[128 * 78 + 128 + 128 * 128 + 128:] *= scale
        dg.dg_mlp_set_params(m, pp)
        qd = pair.to_device(q)
        res = torch.zeros_like(qd)
        dg.dg_run(pair.ctx, qd, res, 4, 0.5, 0.0)
        outs.append(qd.clone())
    assert torch.equal(outs[0], outs[2])
    assert not torch.equal(outs[0], outs[1])
