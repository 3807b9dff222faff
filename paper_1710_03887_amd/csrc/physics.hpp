// Device-side Euler physics in perturbation form (FP32).
//
// The state holds q' = q - q0 (conserved variables minus the ambient state).
// Everything that is formed from q is rewritten so that ambient parts
// cancel analytically, which keeps FP32 accurate for acoustic amplitudes:
//   u - u0 = (m' - rho' u0)/rho,
//   rho|u|^2 - rho0|u0|^2 = m.(u - u0) + m'.u0,
//   p' = (gamma-1) (E' - (rho|u|^2 - rho0|u0|^2)/2)          (Eq. 2),
//   F'_d = ( m'_d,  m_i (u_d - u0_d) + m'_i u0_d + delta_id p',
//            (u_d - u0_d)(E + p) + u0_d (E' + p') )            (Eq. 1).
#pragma once

#include <hip/hip_runtime.h>

namespace dg {

struct Phys {
  float gamma, gm1;
  float rho0, p0, c0, Z0, inv_c0sq;
  float u0[3], m0[3];
  float E0;
  float amp;     // inflow pulse amplitude
  float half_N1sq;  // (N+1)^2 / 2 for the time-step rule
  double alpha;  // inflow pulse angular frequency
};

struct Prim {
  float rho, rhop;   // rho, rho'
  float m[3], mp[3]; // momentum, momentum perturbation
  float du[3];       // u - u0
  float p, pp;       // p, p'
  float E, Ep;       // E, E'
};

// MOVING = false specializes everything below to an ambient state at rest
// (u0 = 0), where the ambient-velocity terms vanish identically.
template <bool MOVING = true>
__device__ __forceinline__ void primitive(const Phys& P, const float q[5], Prim& w) {
  if (!MOVING) {
    w.rhop = q[0];
    w.rho = P.rho0 + q[0];
    const float ir = 1.0f / w.rho;
    float kin = 0.0f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      w.mp[d] = q[1 + d];
      w.m[d] = q[1 + d];
      w.du[d] = q[1 + d] * ir;
      kin += w.mp[d] * w.du[d];
    }
    w.Ep = q[4];
    w.E = P.E0 + q[4];
    w.pp = P.gm1 * (q[4] - 0.5f * kin);
    w.p = P.p0 + w.pp;
    return;
  }
  w.rhop = q[0];
  w.rho = P.rho0 + q[0];
  const float ir = 1.0f / w.rho;
  float kin = 0.0f;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    w.mp[d] = q[1 + d];
    w.m[d] = P.m0[d] + q[1 + d];
    w.du[d] = (w.mp[d] - w.rhop * P.u0[d]) * ir;
    kin += w.m[d] * w.du[d] + w.mp[d] * P.u0[d];
  }
  w.Ep = q[4];
  w.E = P.E0 + q[4];
  w.pp = P.gm1 * (q[4] - 0.5f * kin);
  w.p = P.p0 + w.pp;
}

// Flux perturbation along a unit (or any) direction n: n.F(q) - n.F(q0).
template <bool MOVING = true>
__device__ __forceinline__ void normal_flux(const Phys& P, const Prim& w, const float n[3],
                                            float f[5]) {
  if (!MOVING) {
    const float dun = w.du[0] * n[0] + w.du[1] * n[1] + w.du[2] * n[2];
    f[0] = w.mp[0] * n[0] + w.mp[1] * n[1] + w.mp[2] * n[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) f[1 + i] = w.mp[i] * dun + n[i] * w.pp;
    f[4] = dun * (w.E + w.p);
    return;
  }
  const float dun = w.du[0] * n[0] + w.du[1] * n[1] + w.du[2] * n[2];
  const float u0n = P.u0[0] * n[0] + P.u0[1] * n[1] + P.u0[2] * n[2];
  f[0] = w.mp[0] * n[0] + w.mp[1] * n[1] + w.mp[2] * n[2];
#pragma unroll
  for (int i = 0; i < 3; ++i) f[1 + i] = w.m[i] * dun + w.mp[i] * u0n + n[i] * w.pp;
  f[4] = dun * (w.E + w.p) + u0n * (w.Ep + w.pp);
}

// |u.n| + c
template <bool MOVING = true>
__device__ __forceinline__ float normal_speed(const Phys& P, const Prim& w, const float n[3]) {
  if (!MOVING)
    return fabsf(w.du[0] * n[0] + w.du[1] * n[1] + w.du[2] * n[2]) + sqrtf(P.gamma * w.p / w.rho);
  const float un = (P.u0[0] + w.du[0]) * n[0] + (P.u0[1] + w.du[1]) * n[1] +
                   (P.u0[2] + w.du[2]) * n[2];
  return fabsf(un) + sqrtf(P.gamma * w.p / w.rho);
}

// conserved perturbation from (rho', u - u0, p')
__device__ __forceinline__ void state_from(const Phys& P, float rhop, const float du[3], float pp,
                                           float q[5]) {
  const float rho = P.rho0 + rhop;
  float kin = 0.0f;
  q[0] = rhop;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float mp = rhop * P.u0[d] + rho * du[d];
    const float m = P.m0[d] + mp;
    q[1 + d] = mp;
    kin += m * du[d] + mp * P.u0[d];
  }
  q[4] = pp / P.gm1 + 0.5f * kin;
}

enum : int { BC_INTERIOR = 0, BC_OUTFLOW_CHAR = 1, BC_PASSTHRU = 2, BC_WALL = 3,
             BC_INFLOW = 4, BC_LEARNED = 5 };

// Ghost state q+' for boundary tag `tag`, from the interior trace (qm, w).
__device__ __forceinline__ void ghost(const Phys& P, int tag, const float qm[5], const Prim& w,
                                      const float n[3], float inflow_pp, float qg[5]) {
  if (tag == BC_PASSTHRU) {
#pragma unroll
    for (int v = 0; v < 5; ++v) qg[v] = 0.0f;
  } else if (tag == BC_WALL) {
    const float mn = w.m[0] * n[0] + w.m[1] * n[1] + w.m[2] * n[2];
    qg[0] = qm[0];
#pragma unroll
    for (int d = 0; d < 3; ++d) qg[1 + d] = qm[1 + d] - 2.0f * mn * n[d];
    qg[4] = qm[4];
  } else if (tag == BC_INFLOW) {
    const float pg = inflow_pp;
    const float rhop = P.rho0 * expm1f(log1pf(pg / P.p0) / P.gamma);
    const float s = pg / P.Z0;
    const float du[3] = {-s * n[0], -s * n[1], -s * n[2]};
    state_from(P, rhop, du, pg, qg);
  } else {  // characteristic outflow (also the learned tag without a network)
    const float vn = w.du[0] * n[0] + w.du[1] * n[1] + w.du[2] * n[2];
    const float s = w.rhop - w.pp * P.inv_c0sq;
    const float pg = 0.5f * (w.pp + P.Z0 * vn);
    const float vng = pg / P.Z0;
    float du[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) du[d] = w.du[d] - vn * n[d] + vng * n[d];
    state_from(P, pg * P.inv_c0sq + s, du, pg, qg);
  }
}

}  // namespace dg
