// Right-hand side of curved (isoparametric) elements, the remedy Section 3
// names for the reflections it sees from a spherical boundary built of flat
// faces: the nodal strong form with the metric terms of each node and the
// normal and sJ/J of each face node (the volume term in chain-rule form,
// sum_a sum_d (d r_a/d x_d) D_a F_d, which reduces to the straight-sided
// operator of Appendix A, Eq. 10, for constant metric terms).
//
// One wavefront per curved element (four per block); each wavefront stages
// its element's state, the three Cartesian flux perturbations of every node
// and the face jumps in its own LDS slice and synchronizes only itself.  The
// volume contraction G[(a, n)][(d, v)] = sum_j D_a[n][j] F_dv[j] is one dense
// product, [3 Np x Np] x [Np x 15], on MFMA f32 16x16x4 (the operator packed
// on the host in the instruction's lane order); each node's lane then applies
// its nine metric terms.  Curved elements are the boundary layer of a curved
// outer surface, a small share of the mesh, so one element per wavefront
// (rather than the stage kernel's tiles) keeps this pass simple; its time is
// the latency of each element's chain of phases.
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

__global__ __launch_bounds__(256) void curved_save_kernel(CurvedSet cv, int ST,
                                                          const float* __restrict__ res) {
  const int64_t total = cv.n * ST;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t c = i / ST;
    cv.res_save[i] = res[cv.elem[c] * ST + (i - c * ST)];
  }
}

template <int N, bool MOVING>
__global__ __launch_bounds__(64 * kWavesC) void curved_kernel(
    DeviceMesh m, CurvedSet cv, int mode, const float* __restrict__ q_in, float* __restrict__ q_out,
    float* __restrict__ res, float* __restrict__ out, float a_rk, float b_rk, double c_rk,
    double t_host, double dt_host, const RunScalars* run) {
  constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  constexpr int Nfp = (N + 1) * (N + 2) / 2;
  constexpr int NF = 4 * Nfp, ST = 5 * Np;
  // MFMA tiling of the volume product: MT row tiles of (a, n), KS steps of 4 nodes
  constexpr int MT = (3 * Np + 15) / 16, KS = (Np + 3) / 4;
  // per-wavefront slice, 16-byte aligned regions; the product's rows (sG)
  // reuse the space of the fluxes and face scratch, dead by then
  constexpr int oD = (ST + 3) / 4 * 4, oF = oD + 8 * NF, oQ = oF + 16 * 4 * KS, oS = oQ + 5 * NF;
  constexpr int scratch = (oS + NF - oF) > 16 * 16 * MT ? (oS + NF - oF) : 16 * 16 * MT;
  constexpr int kSlice = (oF + scratch + 3) / 4 * 4;
  __shared__ __align__(16) float lds[kWavesC * kSlice];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t ic = int64_t(blockIdx.x) * kWavesC + w;
  if (ic >= cv.n) return;  // whole wavefront; no block-wide barrier below
  const int64_t k = cv.elem[ic];
  float* sq = lds + w * kSlice;  // [5][Np] state q'
  float* sdF = sq + oD;          // [NF][8]: n.(F- - F+), then the lifted jump (padded)
  float* sF = sq + oF;           // [4 KS][16]: [3 (x,y,z)][5] flux perturbations, zero padded
  float* sdQ = sq + oQ;          // [NF][5] q- - q+
  float* sS = sq + oS;           // [NF] max(|u.n| + c) of both sides
  float* sG = sq + oF;           // [16 MT][16]: the volume product (after the MFMAs)
  const Phys& P = m.phys;
  const double tst = run ? run->t + c_rk * run->dt : t_host + c_rk * dt_host;
  const float pin = pulse_pressure(P, tst);
  const float dt = float(run ? run->dt : dt_host);

  for (int i = lane; i < ST; i += 64) sq[i] = q_in[k * ST + i];
  // zero padding of the flux rows: rows Np .. 4 KS - 1 and column 15
  for (int i = lane; i < 16 * 4 * KS; i += 64)
    if (i >= 16 * Np || (i & 15) == 15) sF[i] = 0.0f;
  wave_sync();
  for (int n = lane; n < Np; n += 64) {
    float qq[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) qq[v] = sq[v * Np + n];
    Prim wv;
    primitive<MOVING>(P, qq, wv);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float e[3] = {d == 0 ? 1.0f : 0.0f, d == 1 ? 1.0f : 0.0f, d == 2 ? 1.0f : 0.0f};
      float f[5];
      normal_flux<MOVING>(P, wv, e, f);
#pragma unroll
      for (int v = 0; v < 5; ++v) sF[n * 16 + d * 5 + v] = f[v];
    }
  }
  // face jumps at every face node, with that node's own normal
  for (int i = lane; i < NF; i += 64) {
    const int f = i / Nfp, ii = i - f * Nfp;
    const int node = m.fmask[i];
    const float* gs = cv.sg + (ic * NF + i) * 4;
    const float nn[3] = {gs[0], gs[1], gs[2]};
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
      sdF[i * 8 + v] = fm[v] - fp[v];
      sdQ[i * 5 + v] = qm[v] - qp[v];
    }
  }
  wave_sync();
  // local Lax-Friedrichs jump, one lambda per face, scaled by the node's sJ/J
  for (int i = lane; i < NF; i += 64) {
    const int f = i / Nfp;
    float lam = 0.0f;
    for (int j = 0; j < Nfp; ++j) lam = fmaxf(lam, sS[f * Nfp + j]);
    const float fs = cv.sg[(ic * NF + i) * 4 + 3];
#pragma unroll
    for (int v = 0; v < 5; ++v) sdF[i * 8 + v] = 0.5f * fs * (sdF[i * 8 + v] - lam * sdQ[i * 5 + v]);
  }
  wave_sync();
  // volume product on MFMA: lane l supplies A[row l%16][k l/16] (packed) and
  // B[k l/16][col l%16] = F of node 4 ks + l/16, column l%16; it holds
  // D[rows 4 (l/16) .. +3][col l%16] of each row tile
  {
    floatx4 acc[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) acc[t] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    const float* Ap = cv.D + lane;
#pragma unroll 3
    for (int ks = 0; ks < KS; ++ks) {
      const float b = sF[(4 * ks + (lane >> 4)) * 16 + (lane & 15)];
#pragma unroll
      for (int t = 0; t < MT; ++t)
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(Ap[(ks * MT + t) * 64], b, acc[t], 0, 0, 0);
    }
    wave_sync();  // every lane is done with the fluxes: sG reuses their space
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) sG[(16 * t + 4 * (lane >> 4) + i) * 16 + (lane & 15)] = acc[t][i];
  }
  wave_sync();
  for (int n = lane; n < Np; n += 64) {
    float G[3][3][5];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float4 g4 = reinterpret_cast<const float4*>(sG + (a * Np + n) * 16)[c];
        const float gv[4] = {g4.x, g4.y, g4.z, g4.w};
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (4 * c + u < 15) G[a][(4 * c + u) / 5][(4 * c + u) % 5] = gv[u];
      }
    }
    const float* g = cv.vg + (ic * Np + n) * 9;
    float gm[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) gm[i] = g[i];
    float r[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      float div = 0.0f;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int d = 0; d < 3; ++d) div += gm[a * 3 + d] * G[a][d][v];
      r[v] = -div;
    }
#pragma unroll 6
    for (int i = 0; i < NF; ++i) {
      const float l = cv.L[size_t(i) * Np + n];
      const float4 d4 = *reinterpret_cast<const float4*>(sdF + i * 8);
      r[0] += l * d4.x;
      r[1] += l * d4.y;
      r[2] += l * d4.z;
      r[3] += l * d4.w;
      r[4] += l * sdF[i * 8 + 4];
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
        const float prev = a_rk != 0.0f ? cv.res_save[ic * ST + v * Np + n] : 0.0f;
        const float rr = dt * r[v] + a_rk * prev;
        res[gi] = rr;
        q_out[gi] = sq[v * Np + n] + b_rk * rr;
      }
    }
  }
}

template <int N>
hipError_t curved_dispatch(const CurvedSet& cv, const DeviceMesh& m, int mode, const float* q_in,
                           float* q_out, float* res, float* out, float a, float b, double c,
                           double t_host, double dt_host, const RunScalars* run, hipStream_t s) {
  const int blocks = int((cv.n + kWavesC - 1) / kWavesC);
  const bool moving = m.phys.u0[0] != 0.0f || m.phys.u0[1] != 0.0f || m.phys.u0[2] != 0.0f;
  if (moving)
    curved_kernel<N, true><<<blocks, 64 * kWavesC, 0, s>>>(m, cv, mode, q_in, q_out, res, out, a, b,
                                                           c, t_host, dt_host, run);
  else
    curved_kernel<N, false><<<blocks, 64 * kWavesC, 0, s>>>(m, cv, mode, q_in, q_out, res, out, a, b,
                                                            c, t_host, dt_host, run);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_curved_save(const CurvedSet& cv, const DeviceMesh& m, const float* res,
                              hipStream_t s) {
  if (cv.n <= 0) return hipSuccess;
  const int64_t total = cv.n * 5 * m.Np;
  const int blocks = int(std::min<int64_t>((total + 255) / 256, 4096));
  curved_save_kernel<<<blocks, 256, 0, s>>>(cv, 5 * m.Np, res);
  return hipGetLastError();
}

hipError_t launch_curved(const CurvedSet& cv, const DeviceMesh& m, int mode, const float* q_in,
                         float* q_out, float* res, float* out, float a, float b, double c,
                         double t_host, double dt_host, const RunScalars* run, hipStream_t s) {
  if (cv.n <= 0) return hipSuccess;
  switch (m.N) {
    case 1: return curved_dispatch<1>(cv, m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, s);
    case 2: return curved_dispatch<2>(cv, m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, s);
    case 3: return curved_dispatch<3>(cv, m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, s);
    case 4: return curved_dispatch<4>(cv, m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, s);
    case 5: return curved_dispatch<5>(cv, m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dg
