// Right-hand side of curved (isoparametric) elements, the remedy Section 3
// names for the reflections it sees from a spherical boundary built of flat
// faces: the nodal strong form with the metric terms of each node and the
// normal and sJ/J of each face node (the volume term in chain-rule form,
// sum_a sum_d (d r_a/d x_d) D_a F_d, which reduces to the straight-sided
// operator of Appendix A, Eq. 10, for constant metric terms).
//
// One wavefront per curved element (four per block); each wavefront stages
// its element's state and the three Cartesian flux perturbations of every
// node in its own LDS slice and synchronizes only itself.  The volume
// contraction G_a[n][(d, v)] = sum_j D_a[n][j] F_dv[j] runs on MFMA f32
// 16x16x4 one direction a at a time ([Np x Np] x [Np x 15], the operator
// packed on the host in the instruction's lane order, the flux operand held
// in registers); after each, the lane of node n applies its metric terms
// d r_a / d x_d.  The face jumps stay in registers until their one-per-face
// Lax-Friedrichs speed is known.  The slice is 5.2 KB at N = 4 (seven
// wavefronts per SIMD).  Curved elements are a small share of the mesh, so
// one element per wavefront (rather than the stage kernel's tiles) keeps
// this pass simple.
#include "curved.hpp"

#include <algorithm>

#include "physics.hpp"

namespace dg {
namespace {

constexpr int kWavesC = 4;

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float pulse_pressure(const Phys& P, double t) {
  const double T = 2.0 * M_PI / P.alpha;
  if (t >= 0.0 && t < T) return float(0.5 * P.amp * (1.0 - cos(P.alpha * t)));
  return 0.0f;
}

template <int N, bool MOVING>
__global__ __launch_bounds__(64 * kWavesC) void curved_kernel(
    DeviceMesh m, CurvedSet cv, int mode, const float* __restrict__ q_in, float* __restrict__ q_out,
    float* __restrict__ res, float* __restrict__ out, float a_rk, float b_rk, double c_rk,
    double t_host, double dt_host, RunScalars* run, int rate_out) {
  constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  constexpr int Nfp = (N + 1) * (N + 2) / 2;
  constexpr int NF = 4 * Nfp, ST = 5 * Np;
  static_assert(Np <= 64, "one node per lane");
  // MFMA tiling of each direction's product: MT row tiles of n, KS steps of 4 nodes
  constexpr int MT = (Np + 15) / 16, KS = (Np + 3) / 4;
  constexpr int NFL = (NF + 63) / 64;   // face nodes per lane
  // per-wavefront slice (floats): state [5][Np] | lifted jumps [5][NF] |
  // fluxes [4 KS][16], later one direction's product [16 MT][16] | face speeds
  constexpr int oD = (ST + 3) / 4 * 4, oF = (oD + 5 * NF + 3) / 4 * 4;
  constexpr int fg = 16 * 4 * KS > 16 * 16 * MT ? 16 * 4 * KS : 16 * 16 * MT;
  constexpr int oS = oF + fg;
  constexpr int kSlice = (oS + NF + 3) / 4 * 4;
  __shared__ __align__(16) float lds[kWavesC * kSlice];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t ic = int64_t(blockIdx.x) * kWavesC + w;
  if (ic >= cv.n) return;  // whole wavefront; no block-wide barrier below
  const int64_t k = cv.elem[ic];
  float* sq = lds + w * kSlice;  // [5][Np] state q'
  float* sdF = sq + oD;          // [5][NF] lifted jumps
  float* sF = sq + oF;           // [4 KS][16]: [3 (x,y,z)][5] flux perturbations, zero padded
  float* sG = sq + oF;           // [16 MT][16]: one direction's product (after the fluxes)
  float* sS = sq + oS;           // [NF] max(|u.n| + c) of both sides
  const Phys& P = m.phys;
  const double tst = run ? run->t + c_rk * run->dt : t_host + c_rk * dt_host;
  const float pin = pulse_pressure(P, tst);
  const float dt = float(run ? run->dt : dt_host);

  for (int i = lane; i < ST; i += 64) sq[i] = q_in[k * ST + i];
  // zero padding of the flux rows: rows Np .. 4 KS - 1 and column 15
  for (int i = lane; i < 16 * 4 * KS; i += 64)
    if (i >= 16 * Np || (i & 15) == 15) sF[i] = 0.0f;
  wave_sync();
  if (lane < Np) {
    float qq[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) qq[v] = sq[v * Np + lane];
    Prim wv;
    primitive<MOVING>(P, qq, wv);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float e[3] = {d == 0 ? 1.0f : 0.0f, d == 1 ? 1.0f : 0.0f, d == 2 ? 1.0f : 0.0f};
      float f[5];
      normal_flux<MOVING>(P, wv, e, f);
#pragma unroll
      for (int v = 0; v < 5; ++v) sF[lane * 16 + d * 5 + v] = f[v];
    }
  }
  // face jumps at every face node, with that node's own normal (kept in
  // registers until the face's speed is reduced)
  float dFr[NFL][5], dQr[NFL][5], fsr[NFL];
#pragma unroll
  for (int it = 0; it < NFL; ++it) {
    const int i = lane + 64 * it;
#pragma unroll
    for (int v = 0; v < 5; ++v) dFr[it][v] = dQr[it][v] = 0.0f;
    fsr[it] = 0.0f;
    if (i >= NF) continue;
    const int f = i / Nfp, ii = i - f * Nfp;
    const int node = m.fmask[i];
    const float4 gs = reinterpret_cast<const float4*>(cv.sg)[ic * NF + i];
    const float nn[3] = {gs.x, gs.y, gs.z};
    fsr[it] = gs.w;
    float qm[5], qp[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) qm[v] = sq[v * Np + node];
    Prim wm, wp;
    primitive<MOVING>(P, qm, wm);
    const int nb = m.nbr[k * 4 + f];
    if (nb >= 0) {
      const int inf = m.finfo[k * 4 + f];
      const int node2 = m.nbr_node[((f * 4 + (inf & 3)) * 6 + (inf >> 2)) * Nfp + ii];
#pragma unroll
      for (int v = 0; v < 5; ++v) qp[v] = q_in[int64_t(nb) * ST + v * Np + node2];
    } else {
      ghost(P, (-nb) & 7, qm, wm, nn, pin, qp);
    }
    primitive<MOVING>(P, qp, wp);
    float fm[5], fp[5];
    normal_flux<MOVING>(P, wm, nn, fm);
    normal_flux<MOVING>(P, wp, nn, fp);
    sS[i] = fmaxf(normal_speed<MOVING>(P, wm, nn), normal_speed<MOVING>(P, wp, nn));
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      dFr[it][v] = fm[v] - fp[v];
      dQr[it][v] = qm[v] - qp[v];
    }
  }
  wave_sync();
  // local Lax-Friedrichs jump, one lambda per face, scaled by the node's sJ/J
#pragma unroll
  for (int it = 0; it < NFL; ++it) {
    const int i = lane + 64 * it;
    if (i >= NF) continue;
    const int f = i / Nfp;
    float lam = 0.0f;
    for (int j = 0; j < Nfp; ++j) lam = fmaxf(lam, sS[f * Nfp + j]);
#pragma unroll
    for (int v = 0; v < 5; ++v) sdF[v * NF + i] = 0.5f * fsr[it] * (dFr[it][v] - lam * dQr[it][v]);
  }
  // B operand of the volume products: lane l holds F of node 4 ks + l/16,
  // column l%16, for every step ks
  float bv[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) bv[ks] = sF[(4 * ks + (lane >> 4)) * 16 + (lane & 15)];
  wave_sync();  // every lane holds its operand: sG reuses the fluxes' space
  const float* g = cv.vg + (ic * Np + (lane < Np ? lane : 0)) * 9;
  float gm[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) gm[i] = lane < Np ? g[i] : 0.0f;
  float r[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    // G_a = D_a F: lane l supplies A[row l%16][k l/16] (packed) and holds
    // rows 4 (l/16) .. +3, column l%16, of each row tile
    floatx4 acc[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) acc[t] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    const float* Ap = cv.D + size_t(a) * KS * MT * 64 + lane;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int t = 0; t < MT; ++t)
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(Ap[(ks * MT + t) * 64], bv[ks], acc[t], 0, 0, 0);
    if (a > 0) wave_sync();  // the previous direction's rows are read
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) sG[(16 * t + 4 * (lane >> 4) + i) * 16 + (lane & 15)] = acc[t][i];
    wave_sync();
    if (lane < Np) {
      // r_v -= sum_d (d r_a / d x_d) G_a[n][(d, v)]
      float G[16];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float4 g4 = reinterpret_cast<const float4*>(sG + lane * 16)[c];
        G[4 * c] = g4.x;
        G[4 * c + 1] = g4.y;
        G[4 * c + 2] = g4.z;
        G[4 * c + 3] = g4.w;
      }
#pragma unroll
      for (int v = 0; v < 5; ++v)
#pragma unroll
        for (int d = 0; d < 3; ++d) r[v] -= gm[a * 3 + d] * G[d * 5 + v];
    }
  }
  const int n = lane;
  if (n < Np) {
#pragma unroll 6
    for (int i = 0; i < NF; ++i) {
      const float l = cv.L[size_t(i) * Np + n];
#pragma unroll
      for (int v = 0; v < 5; ++v) r[v] += l * sdF[v * NF + i];
    }
    if (m.sigma) {
      const float sgm = m.sigma[k * Np + n];
#pragma unroll
      for (int v = 0; v < 5; ++v) r[v] -= sgm * sq[v * Np + n];
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const int64_t gi = k * ST + v * Np + n;
      if (mode == MODE_RHS) {
        out[gi] = r[v];
      } else {
        // the stage kernel leaves the element's residual in place
        const float prev = a_rk != 0.0f ? res[gi] : 0.0f;
        const float rr = dt * r[v] + a_rk * prev;
        const float qn = sq[v * Np + n] + b_rk * rr;
        res[gi] = rr;
        q_out[gi] = qn;
        sq[v * Np + n] = qn;   // (this lane's own node)
      }
    }
  }
  if (mode != MODE_STAGE || !run || !rate_out) return;
  // the element's share of the next time-step rate, from its new state: max
  // over face nodes of (N+1)^2/2 Fscale (|u| + c), Fscale of the
  // straight-sided element (as for every other element)
  wave_sync();
  float best = 0.0f;
  unsigned bad = 0u;
#pragma unroll
  for (int it = 0; it < NFL; ++it) {
    const int i = lane + 64 * it;
    if (i >= NF) continue;
    const int f = i / Nfp, node = m.fmask[i];
    float qq[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) qq[v] = sq[v * Np + node];
    Prim wv;
    primitive<MOVING>(P, qq, wv);
    float sp2 = 0.0f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float u = P.u0[d] + wv.du[d];
      sp2 += u * u;
    }
    const float rate = P.half_N1sq * float(m.sgeo[k * 16 + f * 4 + 3]) *
                       (sqrtf(sp2) + sqrtf(P.gamma * wv.p / wv.rho));
    if (!(wv.rho > 0.0f) || !(wv.p > 0.0f) || !(rate == rate)) bad = 1u;
    else best = fmaxf(best, rate);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    best = fmaxf(best, __shfl_xor(best, off));
    bad |= __shfl_xor(bad, off);
  }
  if (lane == 0) {
    // thousands of small blocks: spread over the run's rate slots
    atomicMax(&run->rate_part[ic & (kRateParts - 1)], __float_as_uint(best));
    if (bad) atomicOr(&run->bad, 1u);
  }
}

template <int N>
hipError_t curved_dispatch(const CurvedSet& cv, const DeviceMesh& m, int mode, const float* q_in,
                           float* q_out, float* res, float* out, float a, float b, double c,
                           double t_host, double dt_host, RunScalars* run, int rate_out,
                           hipStream_t s) {
  const int blocks = int((cv.n + kWavesC - 1) / kWavesC);
  const bool moving = m.phys.u0[0] != 0.0f || m.phys.u0[1] != 0.0f || m.phys.u0[2] != 0.0f;
  if (moving)
    curved_kernel<N, true><<<blocks, 64 * kWavesC, 0, s>>>(m, cv, mode, q_in, q_out, res, out, a, b,
                                                           c, t_host, dt_host, run, rate_out);
  else
    curved_kernel<N, false><<<blocks, 64 * kWavesC, 0, s>>>(m, cv, mode, q_in, q_out, res, out, a, b,
                                                            c, t_host, dt_host, run, rate_out);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_curved(const CurvedSet& cv, const DeviceMesh& m, int mode, const float* q_in,
                         float* q_out, float* res, float* out, float a, float b, double c,
                         double t_host, double dt_host, RunScalars* run, int rate_out,
                         hipStream_t s) {
  if (cv.n <= 0) return hipSuccess;
  switch (m.N) {
    case 1: return curved_dispatch<1>(cv, m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, rate_out, s);
    case 2: return curved_dispatch<2>(cv, m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, rate_out, s);
    case 3: return curved_dispatch<3>(cv, m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, rate_out, s);
    case 4: return curved_dispatch<4>(cv, m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, rate_out, s);
    case 5: return curved_dispatch<5>(cv, m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, rate_out, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dg
