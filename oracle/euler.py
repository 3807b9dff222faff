"""Semi-discrete right-hand side f(c) for the 3D Euler equations (oracle).

State: conserved variables q[K, 5, Np] = (rho, rho u, rho v, rho w, E) at
the nodes of each element, FP64, full values (not perturbations).

Physics (Section 2.1): Eq. 1 with the standard Euler flux (pressure only on
the diagonal momentum entries; the paper's "P" is p) and the ideal-gas law
of Eq. 2.

Discretization (Appendix A, Eqs. 10-12, in strong nodal form):
    dq/dt = -(Dr Fr + Ds Fs + Dt Ft) + sum_f Fscale_f LIFT_f dF_f,
with contravariant fluxes Fr = r_x F + r_y G + r_z H (likewise Fs, Ft) and
the face jump of the local Lax-Friedrichs flux (Section 1.1)
    dF = 1/2 [ n.(F- - F+) - lambda (q- - q+) ],
lambda being the largest |u.n|+c over the face's nodes on both sides.

Ghost states q+ on boundary faces, by tag:
  1 characteristic outflow: the incoming acoustic characteristic is set to
    the ambient value, everything else comes from inside; with p'=p-p0,
    vn=(v-v0).n, Z0=rho0 c0:  p'_g = (p'- + Z0 vn-)/2, vn_g = p'_g/Z0,
    entropy rho'-p'/c0^2 and tangential velocity kept from inside;
  2 pass-through: the ambient rest state (Section 2.2);
  3 reflective wall: density and pressure kept, velocity mirrored about the
    face normal (Section 2.3, Eq. 4, read as v - 2 (v.n) n);
  4 inflow: the raised-cosine pulse p1 of Section 2.4 with amplitude A,
    density from the adiabatic law (Eq. 6, rho0 (p/p0)^(1/gamma)) and the
    inflow velocity from the linear impedance relation (Eq. 5), directed
    into the domain (Eq. 7);
  5 learned closure: a callable maps interior traces to ghost states.
"""
import numpy as np

INTERIOR, OUTFLOW_CHAR, PASSTHRU, WALL, INFLOW, LEARNED = range(6)


class Physics:
    """gamma, ambient state (rho0, u0, p0) and inflow pulse (amp, alpha)."""

    def __init__(self, gamma=1.4, rho0=1.0, u0=(0.0, 0.0, 0.0), p0=1.0 / 1.4,
                 amp=0.0, alpha=2 * np.pi * 565.0 / 343.0):
        self.gamma = float(gamma)
        self.rho0 = float(rho0)
        self.u0 = np.array(u0, dtype=np.float64)
        self.p0 = float(p0)
        self.amp = float(amp)
        self.alpha = float(alpha)
        self.c0 = np.sqrt(self.gamma * self.p0 / self.rho0)
        self.q0 = conserved(np.array([self.rho0, *self.u0, self.p0]), self.gamma)


def conserved(prim, gamma):
    """(rho, u, v, w, p) on the last axis -> (rho, rho u, rho v, rho w, E),
    E = p/(gamma-1) + rho |u|^2 / 2 (Eq. 2)."""
    prim = np.asarray(prim, dtype=np.float64)
    rho = prim[..., 0]
    u = prim[..., 1:4]
    p = prim[..., 4]
    out = np.empty_like(prim)
    out[..., 0] = rho
    out[..., 1:4] = rho[..., None] * u
    out[..., 4] = p / (gamma - 1.0) + 0.5 * rho * np.sum(u * u, axis=-1)
    return out


def primitive(q, gamma):
    """Conserved on the last axis -> (rho, u, v, w, p)."""
    rho = q[..., 0]
    u = q[..., 1:4] / rho[..., None]
    p = (gamma - 1.0) * (q[..., 4] - 0.5 * rho * np.sum(u * u, axis=-1))
    out = np.empty_like(q)
    out[..., 0] = rho
    out[..., 1:4] = u
    out[..., 4] = p
    return out


def flux(q, gamma):
    """Euler flux along each Cartesian direction: [3, ..., 5] for q [..., 5]
    (Eq. 1): F_d = (rho u_d, rho u u_d + p e_d, u_d (E + p))."""
    w = primitive(q, gamma)
    u, p = w[..., 1:4], w[..., 4]
    out = np.empty((3,) + q.shape)
    for d in range(3):
        out[d, ..., 0] = q[..., 1 + d]
        for i in range(3):
            out[d, ..., 1 + i] = q[..., 1 + i] * u[..., d]
        out[d, ..., 1 + d] += p
        out[d, ..., 4] = u[..., d] * (q[..., 4] + p)
    return out


def normal_flux(q, n, gamma):
    """n . F(q) for q [..., 5] and unit normals n [..., 3]."""
    F = flux(q, gamma)
    return np.einsum("d...v,...d->...v", F, n)


def sound_speed(q, gamma):
    w = primitive(q, gamma)
    return np.sqrt(gamma * w[..., 4] / w[..., 0])


def inflow_pressure(phys, t):
    """Raised-cosine pulse of Section 2.4: p0 + A (1 - cos(alpha t))/2 for
    0 <= t < 2 pi/alpha, else p0 (A = 0.1 p0 gives the paper's p1)."""
    if 0.0 <= t < 2 * np.pi / phys.alpha:
        return phys.p0 + phys.amp * 0.5 * (1.0 - np.cos(phys.alpha * t))
    return phys.p0


def ghost_state(tag, qm, n, phys, t, learned=None):
    """Ghost conserved state for interior traces qm [..., 5], normals n [..., 3]."""
    g = phys.gamma
    if tag == PASSTHRU:
        return np.broadcast_to(phys.q0, qm.shape).copy()
    if tag == WALL:
        w = primitive(qm, g)
        u = w[..., 1:4]
        un = np.sum(u * n, axis=-1)
        w[..., 1:4] = u - 2.0 * un[..., None] * n
        return conserved(w, g)
    if tag == OUTFLOW_CHAR:
        w = primitive(qm, g)
        c0, rho0, p0 = phys.c0, phys.rho0, phys.p0
        Z0 = rho0 * c0
        dv = w[..., 1:4] - phys.u0
        vn = np.sum(dv * n, axis=-1)
        vt = dv - vn[..., None] * n
        pp = w[..., 4] - p0
        s = (w[..., 0] - rho0) - pp / c0 ** 2
        wout = pp + Z0 * vn
        pg = 0.5 * wout
        vng = pg / Z0
        out = np.empty_like(w)
        out[..., 0] = rho0 + pg / c0 ** 2 + s
        out[..., 1:4] = phys.u0 + vt + vng[..., None] * n
        out[..., 4] = p0 + pg
        return conserved(out, g)
    if tag == INFLOW:
        ph = inflow_pressure(phys, t)
        out = np.empty(qm.shape)
        out[..., 0] = phys.rho0 * (ph / phys.p0) ** (1.0 / g)
        out[..., 1:4] = phys.u0 - n * (ph - phys.p0) / (phys.rho0 * phys.c0)
        out[..., 4] = ph
        return conserved(out, g)
    if tag == LEARNED:
        if learned is None:
            raise ValueError("learned boundary faces need a closure")
        return learned(qm, n)
    raise ValueError(f"unknown boundary tag {tag}")


def face_traces(mesh, q, t, phys, learned=None):
    """Interior and exterior traces [K, 4, Nfp, 5] and the normals."""
    ref = mesh.ref
    K, Np, Nfp = mesh.K, ref.Np, ref.Nfp
    qn = np.transpose(q, (0, 2, 1))                       # [K, Np, 5]
    qm = qn[:, ref.Fmask, :]                              # [K, 4, Nfp, 5]
    flat = qn.reshape(K * Np, 5)
    qp = np.empty_like(qm)
    inner = mesh.mapP >= 0
    qp[inner] = flat[mesh.mapP[inner]]
    nrm = np.broadcast_to(mesh.normals[:, :, None, :], (K, 4, Nfp, 3))
    for tag in np.unique(mesh.bc[mesh.EToE < 0]):
        sel = (mesh.EToE < 0) & (mesh.bc == tag)          # [K, 4]
        qp[sel] = ghost_state(int(tag), qm[sel], nrm[sel], phys, t, learned)
    return qm, qp, nrm


def rhs(mesh, q, t, phys, learned=None, pointwise_lambda=False, sigma=None):
    """f(q) of Eq. 12 for the whole mesh: returns dq/dt [K, 5, Np].  With
    sigma [K, Np] (an absorbing layer, an addition to the method), every node
    also relaxes towards the ambient state: - sigma (q - q0)."""
    ref = mesh.ref
    g = phys.gamma
    qn = np.transpose(q, (0, 2, 1))                       # [K, Np, 5]
    F = flux(qn, g)                                       # [3, K, Np, 5]
    # contravariant fluxes: Fc[k, a] = sum_d (d r_a / d x_d) F_d
    Fc = np.einsum("kad,dkiv->akiv", mesh.drst_dx, F)     # [3, K, Np, 5]
    div = ref.Dr @ Fc[0] + ref.Ds @ Fc[1] + ref.Dt @ Fc[2]  # [K, Np, 5]

    qm, qp, nrm = face_traces(mesh, q, t, phys, learned)
    fm = normal_flux(qm, nrm, g)
    fp = normal_flux(qp, nrm, g)
    unm = np.abs(np.sum(primitive(qm, g)[..., 1:4] * nrm, axis=-1)) + sound_speed(qm, g)
    unp = np.abs(np.sum(primitive(qp, g)[..., 1:4] * nrm, axis=-1)) + sound_speed(qp, g)
    lam = np.maximum(unm, unp)                            # [K, 4, Nfp]
    if not pointwise_lambda:
        lam = np.broadcast_to(lam.max(axis=2, keepdims=True), lam.shape)
    dF = 0.5 * ((fm - fp) - lam[..., None] * (qm - qp))   # [K, 4, Nfp, 5]
    dF = dF * mesh.Fscale[:, :, None, None]
    lifted = ref.LIFT @ dF.reshape(mesh.K, 4 * ref.Nfp, 5)
    out = np.transpose(-div + lifted, (0, 2, 1)).copy()   # [K, 5, Np]
    if sigma is not None:
        out -= sigma[:, None, :] * (q - phys.q0[None, :, None])
    return out


def initial_state(prim, gamma):
    """Conserved state [K, 5, Np] from primitive fields [K, Np, 5]."""
    return np.transpose(conserved(prim, gamma), (0, 2, 1)).copy()
