"""Pins of the oracle's boundary-closure MLP (forward, loss, backward, Adam)
against facts other than itself: known values of the normal distribution
function, the odd-part identity of x Phi(x), central finite differences,
torch's FP64 autograd as an independent library, and closed forms of the
Adam update."""
import numpy as np
import pytest

from oracle import mlp
from workloads.mlp_init import init_params


def test_gelu_known_values_and_identity():
    # Phi(1) and Phi(2) from tables of the standard normal distribution
    assert abs(mlp.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15
    assert abs(mlp.gelu(np.array(2.0)) - 2 * 0.9772498680518208) < 1e-15
    assert mlp.gelu(np.array(0.0)) == 0.0
    x = np.linspace(-4, 4, 81)
    # x Phi(x) - (-x) Phi(-x) = x (Phi(x) + Phi(-x)) = x
    assert np.max(np.abs(mlp.gelu(x) - mlp.gelu(-x) - x)) < 1e-14


def test_gelu_grad_matches_differences():
    x = np.linspace(-5, 5, 101)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(x))) < 1e-8


def test_param_count_and_layout():
    assert mlp.n_params() == 36299
    p = np.arange(mlp.n_params(), dtype=np.float64)
    (W1, b1), (W2, b2), (W3, b3) = mlp.unpack(p)
    assert W1.shape == (128, 78) and W1[0, 1] == 1 and b1[0] == 128 * 78
    assert W3.shape == (75, 128) and b3[-1] == p[-1]


def test_loss_values():
    rng = np.random.default_rng(0)
    Y = rng.normal(size=(5, 75))
    assert mlp.loss(Y, Y) == 0.0
    # a prediction of zero gives |y|^2 / (|y|^2 + eps) per row
    expect = np.mean(np.sum(Y ** 2, 1) / (np.sum(Y ** 2, 1) + 1e-6))
    assert abs(mlp.loss(np.zeros_like(Y), Y) - expect) < 1e-15


def test_gradient_matches_central_differences():
    sizes = (6, 7, 5, 4)
    rng = np.random.default_rng(1)
    p = init_params(3, sizes) + 0.1 * rng.normal(size=mlp.n_params(sizes))
    X = rng.normal(size=(3, 6))
    Y = rng.normal(size=(3, 4))
    L, g = mlp.grad(p, X, Y, sizes=sizes)
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        Lp = mlp.loss(mlp.forward(p + e, X, sizes)[0], Y)
        Lm = mlp.loss(mlp.forward(p - e, X, sizes)[0], Y)
        fd[i] = (Lp - Lm) / (2 * h)
    assert abs(L - mlp.loss(mlp.forward(p, X, sizes)[0], Y)) < 1e-15
    assert np.max(np.abs(fd - g)) / np.max(np.abs(g)) < 1e-6


def test_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(2)
    p = init_params(0)
    X = rng.normal(size=(16, 78))
    Y = rng.normal(size=(16, 75))
    L, g = mlp.grad(p, X, Y)
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    o, layers = 0, []
    for n_in, n_out in ((78, 128), (128, 128), (128, 75)):
        W = pt[o:o + n_in * n_out].view(n_out, n_in)
        o += n_in * n_out
        b = pt[o:o + n_out]
        o += n_out
        layers.append((W, b))
    a = torch.tensor(X)
    for i, (W, b) in enumerate(layers):
        a = a @ W.T + b
        if i < 2:
            a = torch.nn.functional.gelu(a)
    Yt = torch.tensor(Y)
    Lt = torch.mean(((a - Yt) ** 2).sum(1) / ((Yt ** 2).sum(1) + 1e-6))
    Lt.backward()
    assert abs(Lt.item() - L) < 1e-12 * max(1.0, abs(L))
    assert np.max(np.abs(pt.grad.numpy() - g)) < 1e-12 * np.max(np.abs(g))


def test_adam_closed_forms():
    # with a constant gradient the bias-corrected moments are exactly g and
    # g^2, so every step moves each parameter by -lr g / (|g| + eps)
    g = np.array([3.0, -0.5, 1e-3, -7.0])
    p = np.zeros(4)
    opt = mlp.Adam(4)
    for k in range(5):
        p_new = opt.step(p, g, 1e-2)
        assert np.allclose(p_new - p, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
        p = p_new
    # second step after a sign flip: m = 0.9*0.1*g - 0.1*g
    opt = mlp.Adam(1)
    p1 = opt.step(np.zeros(1), np.array([1.0]), 1.0)
    p2 = opt.step(p1, np.array([-1.0]), 1.0)
    m = 0.9 * 0.1 - 0.1
    v = 0.999 * 0.001 + 0.001
    step = (m / (1 - 0.81)) / (np.sqrt(v / (1 - 0.999 ** 2)) + 1e-8)
    assert abs((p2 - p1)[0] + step) < 1e-14


def test_per_face_scaling_is_amplitude_equivariant():
    """With per-face scaling the network sees the same rows for c * q' as
    for q', so its ghost perturbation scales by exactly c."""
    rng = np.random.default_rng(3)
    dq = rng.normal(size=(6, 5, 15))
    n = rng.normal(size=(6, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    s = mlp.face_scale(dq, 0.0)
    assert np.allclose(s, np.abs(dq.reshape(6, -1)).max(axis=1))
    X1 = mlp.face_inputs(dq, n, s)
    X2 = mlp.face_inputs(1e-3 * dq, n, mlp.face_scale(1e-3 * dq, 0.0))
    assert np.allclose(X1, X2, rtol=1e-13, atol=0)
    assert np.max(np.abs(X1[:, :75])) == 1.0
    # a fixed norm divides every face by the same amplitude
    assert np.allclose(mlp.face_inputs(dq, n, mlp.face_scale(dq, 0.5))[:, :75],
                       dq.reshape(6, -1) / 0.5)
