"""Primitive initial fields (rho, u, v, w, p) evaluated at given points.

These are inputs, not part of the discretization: each consumer converts
them to its own state representation.  Coordinates ``x`` have shape
[..., 3]; every function returns an array [..., 5] of (rho, u, v, w, p).
"""
import numpy as np


def gaussian_pulse(x, amp, width, center=(0.0, 0.0, 0.0), rho0=1.0, p0=1.0 / 1.4,
                   gamma=1.4):
    """Fluid at rest with p = p0 + amp*exp(-|x-c|^2/width^2) and isentropic
    density rho = rho0*(p/p0)^(1/gamma)."""
    x = np.asarray(x, dtype=np.float64)
    r2 = np.sum((x - np.asarray(center)) ** 2, axis=-1)
    p = p0 + amp * np.exp(-r2 / width ** 2)
    rho = rho0 * (p / p0) ** (1.0 / gamma)
    out = np.zeros(x.shape[:-1] + (5,))
    out[..., 0] = rho
    out[..., 4] = p
    return out


def plane_wave(x, t, amp, direction, wavenumber, rho0=1.0, p0=1.0 / 1.4, gamma=1.4,
               phase=0.0):
    """Linear acoustic plane wave travelling along unit ``direction``:
    p' = amp*sin(k (d.x - c0 t) + phase), u' = p'/(rho0 c0) d, rho' = p'/c0^2.
    Exact for the linearized equations about the fluid at rest."""
    x = np.asarray(x, dtype=np.float64)
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    c0 = np.sqrt(gamma * p0 / rho0)
    pp = amp * np.sin(wavenumber * (x @ d - c0 * t) + phase)
    out = np.zeros(x.shape[:-1] + (5,))
    out[..., 0] = rho0 + pp / c0 ** 2
    out[..., 1:4] = (pp / (rho0 * c0))[..., None] * d
    out[..., 4] = p0 + pp
    return out


def isentropic_vortex(x, t, beta=5.0, center=(0.0, 0.0), velocity=(1.0, 1.0),
                      gamma=1.4, period=None):
    """Isentropic vortex in the x-y plane, uniform in z, advected by
    ``velocity``: an exact smooth solution of the Euler equations with
    free-stream rho = p = 1.  With ``period`` (Lx, Ly) the nearest periodic
    image of the centre is used."""
    x = np.asarray(x, dtype=np.float64)
    cx = center[0] + velocity[0] * t
    cy = center[1] + velocity[1] * t
    dx = x[..., 0] - cx
    dy = x[..., 1] - cy
    if period is not None:
        dx = dx - period[0] * np.round(dx / period[0])
        dy = dy - period[1] * np.round(dy / period[1])
    r2 = dx * dx + dy * dy
    e = np.exp(0.5 * (1.0 - r2))
    u = velocity[0] - beta / (2 * np.pi) * dy * e
    v = velocity[1] + beta / (2 * np.pi) * dx * e
    T = 1.0 - (gamma - 1.0) * beta ** 2 / (8 * gamma * np.pi ** 2) * e * e
    rho = T ** (1.0 / (gamma - 1.0))
    out = np.zeros(x.shape[:-1] + (5,))
    out[..., 0] = rho
    out[..., 1] = u
    out[..., 2] = v
    out[..., 4] = rho ** gamma
    return out
