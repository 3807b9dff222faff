"""Pressure probes and amplitude spectra, FP64 -- TEST INFRASTRUCTURE ONLY
(see the package docstring).

Section 3 records the pressure of each simulation at sensor points (Table 2
lists their positions relative to the bell and to the outer boundary) and
compares the signals' frequency content in decibels.  The oracle evaluates
the numerical solution at a point the plain way:

* locate: for every element, solve the 4 x 4 system for the point's
  barycentric coordinates (sum of the vertices weighted by them = the point,
  weights summing to one); the point belongs to the element whose smallest
  coordinate is largest (the first such element on ties);
* interpolate: the nodal polynomial of that element through its nodal values
  (monomial basis: solve V^T w = m(r, s, t) for the weights w, V the monomial
  Vandermonde matrix at the reference nodes, m the monomials at the point),
  applied to each conserved variable;
* pressure: p - p0 of the interpolated conserved state by Eq. 2;
* spectrum: the one-sided amplitude spectrum of a uniformly sampled signal
  from the discrete Fourier transform (numpy.fft.rfft as the transform),
  A_k = 2 |X_k| / n (|X_k| / n at k = 0 and at k = n/2), in dB relative to a
  reference amplitude, floored at -600 dB.
"""
import numpy as np

from .euler import primitive
from .operators import vandermonde


def locate(mesh, points):
    """Element index [n] and reference coordinates [n, 3] of each point, or
    element -1 where the smallest barycentric coordinate is below -1e-9."""
    pts = np.atleast_2d(np.asarray(points, dtype=np.float64))
    X = mesh.xyz                                          # [K, 4, 3], oriented
    A = np.concatenate([np.transpose(X, (0, 2, 1)), np.ones((mesh.K, 1, 4))], axis=1)  # [K, 4, 4]
    elem = np.empty(len(pts), dtype=np.int64)
    rst = np.empty((len(pts), 3))
    for p, x in enumerate(pts):
        rhs = np.broadcast_to(np.append(x, 1.0), (mesh.K, 4))
        lam = np.linalg.solve(A, rhs[..., None])[..., 0]  # [K, 4]
        mins = lam.min(axis=1)
        k = int(np.argmax(mins))
        elem[p] = k if mins[k] >= -1e-9 else -1
        # x = lam0 v0 + lam1 v1 + lam2 v2 + lam3 v3 with lam_a = (1 + r_a) / 2
        rst[p] = 2.0 * lam[k, 1:] - 1.0
    return elem, rst


def weights(ref, rst):
    """Nodal interpolation weights [n, Np] at reference points rst [n, 3]."""
    V = vandermonde(ref.N, ref.rst)[0]                     # [Np nodes, Np monomials]
    m = vandermonde(ref.N, np.atleast_2d(rst))[0]          # [n, Np monomials]
    return np.linalg.solve(V.T, m.T).T


def sample(mesh, q, elem, w, phys):
    """p - p0 at the probes: q [K, 5, Np] conserved (full) state."""
    qi = np.einsum("pi,pvi->pv", w, q[elem])               # [n, 5]
    return primitive(qi, phys.gamma)[:, 4] - phys.p0


def record(mesh, q, phys, nsteps, dt, elem, w, t0=0.0):
    """Advance nsteps with the fixed step dt (LSERK4) and sample after each
    step: (final state, end time, series [nsteps, n])."""
    from .timestep import lserk_step
    from .euler import rhs
    series = np.empty((nsteps, len(elem)))
    t, res = t0, None
    for j in range(nsteps):
        q, res = lserk_step(lambda qq, tt: rhs(mesh, qq, tt, phys), q, t, dt, res)
        t = t + dt
        series[j] = sample(mesh, q, elem, w, phys)
    return q, t, series


def spectrum(x, p_ref):
    """dB amplitude spectra of the columns of x [n_samples, n_signals]:
    [n_signals, n_samples // 2 + 1]."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    X = np.fft.rfft(x, axis=0).T                           # [n_signals, n//2 + 1]
    scale = np.full(X.shape[1], 2.0 / n)
    scale[0] = 1.0 / n
    if n % 2 == 0:
        scale[-1] = 1.0 / n
    a = np.abs(X) * scale
    return 20.0 * np.log10(np.maximum(a, 1e-30 * p_ref) / p_ref)
