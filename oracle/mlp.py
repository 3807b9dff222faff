"""Learned boundary closure: the multilayer perceptron, FP64 -- TEST
INFRASTRUCTURE ONLY (see the package docstring).

The input of a boundary face is its interior trace with the incoming
acoustic characteristic removed -- the characteristic ghost state of the
interior trace, as a perturbation q - q0 at the face's Nfp nodes for all five
conserved variables, divided by a scale -- and its outward unit normal; the
output is the exterior (ghost) trace in the same scale:

    z1 = W1 x + b1,  a1 = gelu(z1),
    z2 = W2 a1 + b2, a2 = gelu(z2),
    y  = W3 a2 + b3,

with gelu(x) = x Phi(x) (Phi the standard normal distribution function).
Sizes at N = 4: 78 -> 128 -> 128 -> 75.  The loss of a minibatch is the mean
relative squared error  |y_hat - y|^2 / (|y|^2 + eps).  Training uses Adam
(Kingma & Ba 2015) with bias correction.

Parameters are one flat vector in the order W1 (row-major, out x in), b1,
W2, b2, W3, b3.  Trace layout inside x and y: variable-major,
x[v * Nfp + i] for variable v at face node i, then the normal (x only).

The closure itself is an addition to the method (the paper's
boundary treatments are the pass-through and characteristic ghosts of
Section 2); nothing here reproduces a formula of the paper.
"""
import numpy as np
from scipy.special import erf

SIZES = (78, 128, 128, 75)


def n_params(sizes=SIZES):
    return sum(sizes[i + 1] * sizes[i] + sizes[i + 1] for i in range(len(sizes) - 1))


def unpack(params, sizes=SIZES):
    """[(W, b)] per layer, views into params."""
    out, o = [], 0
    for i in range(len(sizes) - 1):
        n_in, n_out = sizes[i], sizes[i + 1]
        W = params[o:o + n_out * n_in].reshape(n_out, n_in)
        o += n_out * n_in
        b = params[o:o + n_out]
        o += n_out
        out.append((W, b))
    assert o == params.size
    return out


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def forward(params, X, sizes=SIZES):
    """X [B, n_in] -> (Y [B, n_out], cache of pre-activations and inputs)."""
    layers = unpack(np.asarray(params, dtype=np.float64), sizes)
    a = np.asarray(X, dtype=np.float64)
    cache = []
    for li, (W, b) in enumerate(layers):
        z = a @ W.T + b
        cache.append((a, z))
        a = gelu(z) if li < len(layers) - 1 else z
    return a, cache


def loss(Y_hat, Y, eps=1e-6):
    """Mean over the batch of |y_hat - y|^2 / (|y|^2 + eps)."""
    num = np.sum((Y_hat - Y) ** 2, axis=1)
    den = np.sum(Y ** 2, axis=1) + eps
    return float(np.mean(num / den))


def grad(params, X, Y, eps=1e-6, sizes=SIZES):
    """(loss, dloss/dparams) by the chain rule, layer by layer."""
    params = np.asarray(params, dtype=np.float64)
    layers = unpack(params, sizes)
    Y_hat, cache = forward(params, X, sizes)
    B = Y.shape[0]
    den = np.sum(Y ** 2, axis=1) + eps
    L = float(np.mean(np.sum((Y_hat - Y) ** 2, axis=1) / den))
    d = 2.0 * (Y_hat - Y) / (den[:, None] * B)          # dL/dy_hat
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        a_in, z = cache[li]
        if li < len(layers) - 1:
            d = d * gelu_grad(z)                          # through the activation
        grads.append((d.T @ a_in, d.sum(axis=0)))         # dW = dz^T a, db = sum dz
        d = d @ W                                         # to the layer input
    grads.reverse()
    return L, np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


class Adam:
    """Adam with bias correction; state m, v and step count t."""

    def __init__(self, n, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.beta1, self.beta2, self.eps = beta1, beta2, eps

    def step(self, params, g, lr):
        self.t += 1
        self.m = self.beta1 * self.m + (1 - self.beta1) * g
        self.v = self.beta2 * self.v + (1 - self.beta2) * g * g
        m_hat = self.m / (1 - self.beta1 ** self.t)
        v_hat = self.v / (1 - self.beta2 ** self.t)
        return params - lr * m_hat / (np.sqrt(v_hat) + self.eps)


def face_scale(q_minus, norm):
    """Normalization of each face: the fixed amplitude norm > 0, or (norm = 0)
    the face's largest |q - q0| over the given trace [F, 5, Nfp].  [F]"""
    F = q_minus.shape[0]
    if norm > 0:
        return np.full(F, float(norm))
    return np.abs(q_minus.reshape(F, -1)).max(axis=1)


def face_inputs(q_minus, normals, scale):
    """Network input rows from interior traces q_minus [F, 5, Nfp] (perturbations),
    outward unit normals [F, 3] and per-face scales [F]."""
    F = q_minus.shape[0]
    s = np.broadcast_to(np.asarray(scale, dtype=np.float64), (F,))
    inv = np.where(s > 0, 1.0 / np.where(s > 0, s, 1.0), 0.0)
    return np.concatenate([q_minus.reshape(F, -1) * inv[:, None], normals], axis=1)


def closure(params, phys, norm, amp_range, sizes=SIZES, blend=1.0):
    """Ghost-state callable for `euler.rhs(..., learned=...)`.

    The network's input is the characteristic ghost of the interior trace
    (the interior trace without its incoming acoustic characteristic), so a
    network cannot hand the interior's incoming characteristic straight back
    as the ghost's; norm: > 0 a fixed scale, 0 each face's own (face_scale of
    that input).  Face by face: the network's exterior trace, unless the largest interior
    pressure perturbation |p'| on the face lies outside
    [amp_range[0] / 2, 2 amp_range[1]] (outside the trained window, which
    includes a face the wave has not reached) or the network's state has
    rho <= 0 or p <= 0 at a node; such faces take the characteristic ghost.
    On the others the ghost is char + blend * (network - char).
    qm: conserved interior traces [F, Nfp, 5] in the face-node order of the
    network's features; n: unit normals [F, Nfp, 3].
    """
    from .euler import OUTFLOW_CHAR, ghost_state, primitive
    lo, hi = 0.5 * amp_range[0], 2.0 * amp_range[1]
    g = phys.gamma

    def learned(qm, n):
        F, Nfp = qm.shape[0], qm.shape[1]
        qc = ghost_state(OUTFLOW_CHAR, qm, n, phys, 0.0)
        dc = np.transpose(qc - phys.q0, (0, 2, 1))               # [F, 5, Nfp]
        s = face_scale(dc, norm)
        X = face_inputs(dc, n[:, 0, :], s)
        Y, _ = forward(params, X, sizes)
        qn = phys.q0 + np.transpose(Y.reshape(F, 5, Nfp), (0, 2, 1)) * s[:, None, None]
        qp = qc + blend * (qn - qc)
        pmax = np.max(np.abs(primitive(qm, g)[..., 4] - phys.p0), axis=1)
        wp = primitive(qp, g)
        ok = (pmax >= lo) & (pmax <= hi) & (s > 0)
        ok &= np.all((wp[..., 0] > 0) & (wp[..., 4] > 0), axis=1)
        return np.where(ok[:, None, None], qp, qc)

    return learned
