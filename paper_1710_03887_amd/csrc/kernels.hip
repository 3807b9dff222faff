// HIP kernels of the nodal DG Euler hot path (gfx950 / CDNA4).
//
// One block owns a tile of E = 16 consecutive elements and does, in LDS:
//   1. stage the tile's state q' [E][5][Np] (contiguous, coalesced);
//   2. volume: flux perturbations at every node, contravariant fluxes
//      Fr = r_x F + r_y G + r_z H (likewise Fs, Ft) written as the first
//      3 Np rows of the operand B [KT x 5E] (Appendix A, Eq. 10, volume term);
//   3. surface: interior trace from LDS, exterior trace gathered from the
//      neighbour element (or a ghost state by tag), local Lax-Friedrichs
//      jump dF = [n.(F- - F+) - lambda (q- - q+)]/2 scaled by Fscale, as the
//      last 4 Nfp rows of B (Appendix A, Eq. 10, boundary term);
//   4. one dense contraction rhs = A B with A = [-Dr -Ds -Dt LIFT]
//      (Np x KT), on MFMA f32 16x16x4;
//   5. epilogue: write rhs, or the fused LSERK stage update.
// Elements are element-major in HBM; blocks are mapped so that each of the
// 8 XCDs sweeps a contiguous range of tiles (neighbour traces then tend to
// hit that XCD's L2).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"

namespace dg {
namespace {

constexpr int kTileE = 16;
constexpr int kThreads = 256;

typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int N>
struct Shape {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
  static constexpr int NF = 4 * Nfp;              // face nodes per element
  static constexpr int KT = 3 * Np + NF;          // contraction length
  static constexpr int KT4 = (KT + 3) / 4 * 4;    // padded to the MFMA k-step
  static constexpr int MP = (Np + 15) / 16 * 16;  // rows padded to 16
  static constexpr int MT = MP / 16;
  static constexpr int NCOL = 5 * kTileE;         // columns: (element, variable)
  static constexpr int NT = NCOL / 16;
  static constexpr int ST = 5 * Np;               // floats per element state
  // LDS layout (floats)
  static constexpr int oB = 0;                    // [KT4][NCOL]
  static constexpr int oQ = oB + KT4 * NCOL;      // [E][5][Np]
  static constexpr int oG = oQ + kTileE * ST;     // [E][9] metric
  static constexpr int oS = oG + kTileE * 9;      // [E][4][4] normal + Fscale
  static constexpr int oL = oS + kTileE * 16;     // [E][4] face lambda (bits)
  static constexpr int total = oL + kTileE * 4;
};

__device__ __forceinline__ int tile_of_block(int b, int G) {
  // XCD x (= b mod 8) takes a contiguous range of tiles
  const int x = b & 7, j = b >> 3;
  const int per = G >> 3, rem = G & 7;
  return x * per + (x < rem ? x : rem) + j;
}

__device__ __forceinline__ double stage_time(double c, double t_host, double dt_host,
                                             const RunScalars* run) {
  if (run) return run->t + c * run->dt;
  return t_host + c * dt_host;
}

__device__ __forceinline__ float inflow_pressure(const Phys& P, double t) {
  const double T = 2.0 * M_PI / P.alpha;
  if (t >= 0.0 && t < T) return float(0.5 * P.amp * (1.0 - cos(P.alpha * t)));
  return 0.0f;
}

template <int N, int MODE>
__global__ __launch_bounds__(kThreads) void stage_kernel(DeviceMesh m, const float* __restrict__ q_in,
                                                         float* __restrict__ q_out,
                                                         float* __restrict__ res,
                                                         float* __restrict__ out, float a_rk,
                                                         float b_rk, double c_rk, double t_host,
                                                         double dt_host, const RunScalars* run) {
  using S = Shape<N>;
  extern __shared__ float lds[];
  float* sB = lds + S::oB;
  float* sQ = lds + S::oQ;
  float* sG = lds + S::oG;
  float* sS = lds + S::oS;
  unsigned* sL = reinterpret_cast<unsigned*>(lds + S::oL);
  const Phys& P = m.phys;

  const int G = gridDim.x;
  const int tile = tile_of_block(blockIdx.x, G);
  const int64_t e0 = int64_t(tile) * kTileE;
  const int ne = int(min<int64_t>(kTileE, m.K - e0));
  const int tid = threadIdx.x;

  // 1. stage state and geometry
  const float* qg = q_in + e0 * S::ST;
  if (ne == kTileE) {
    const float4* src = reinterpret_cast<const float4*>(qg);
    float4* dst = reinterpret_cast<float4*>(sQ);
    for (int i = tid; i < kTileE * S::ST / 4; i += kThreads) dst[i] = src[i];
  } else {
    for (int i = tid; i < kTileE * S::ST; i += kThreads) sQ[i] = (i < ne * S::ST) ? qg[i] : 0.0f;
  }
  for (int i = tid; i < kTileE * 9; i += kThreads)
    sG[i] = (i < ne * 9) ? float(m.vgeo[e0 * 9 + i]) : 0.0f;
  for (int i = tid; i < kTileE * 16; i += kThreads)
    sS[i] = (i < ne * 16) ? float(m.sgeo[e0 * 16 + i]) : 0.0f;
  for (int i = tid; i < kTileE * 4; i += kThreads) sL[i] = 0u;
  for (int i = S::KT * S::NCOL + tid; i < S::KT4 * S::NCOL; i += kThreads) sB[i] = 0.0f;
  __syncthreads();

  // 2. volume fluxes -> rows [a*Np + node] of B
  for (int it = tid; it < kTileE * S::Np; it += kThreads) {
    const int e = it / S::Np, i = it - e * S::Np;
    float q[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) q[v] = sQ[e * S::ST + v * S::Np + i];
    Prim w;
    primitive(P, q, w);
    const float* g = sG + e * 9;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      // contravariant direction: grad of reference coordinate ax
      const float n[3] = {g[ax * 3 + 0], g[ax * 3 + 1], g[ax * 3 + 2]};
      float f[5];
      normal_flux(P, w, n, f);
      float* row = sB + (ax * S::Np + i) * S::NCOL + e * 5;
#pragma unroll
      for (int v = 0; v < 5; ++v) row[v] = (e < ne) ? f[v] : 0.0f;
    }
  }

  // 3. surface traces; lambda per face via an LDS max
  constexpr int kFaceIters = (kTileE * S::NF + kThreads - 1) / kThreads;
  float qm[kFaceIters][5], qp[kFaceIters][5];
  const float pin = inflow_pressure(P, stage_time(c_rk, t_host, dt_host, run));
#pragma unroll
  for (int s = 0; s < kFaceIters; ++s) {
    const int it = tid + s * kThreads;
    if (it >= kTileE * S::NF) break;
    const int e = it / S::NF, fi = it - e * S::NF;
    const int f = fi / S::Nfp, i = fi - f * S::Nfp;
    if (e >= ne) {
#pragma unroll
      for (int v = 0; v < 5; ++v) qm[s][v] = qp[s][v] = 0.0f;
      continue;
    }
    const int node = m.fmask[f * S::Nfp + i];
#pragma unroll
    for (int v = 0; v < 5; ++v) qm[s][v] = sQ[e * S::ST + v * S::Np + node];
    const float* sg = sS + e * 16 + f * 4;
    const float n[3] = {sg[0], sg[1], sg[2]};
    Prim wm;
    primitive(P, qm[s], wm);
    const int64_t k = e0 + e;
    const int nb = m.nbr[k * 4 + f];
    if (nb >= 0) {
      const int info = m.finfo[k * 4 + f];
      const int f2 = info & 3, o = info >> 2;
      const int n2 = m.nbr_node[((f * 4 + f2) * 6 + o) * S::Nfp + i];
      const float* qn = q_in + int64_t(nb) * S::ST + n2;
#pragma unroll
      for (int v = 0; v < 5; ++v) qp[s][v] = qn[v * S::Np];
    } else {
      ghost(P, -nb, qm[s], wm, n, pin, qp[s]);
    }
    Prim wp;
    primitive(P, qp[s], wp);
    const float lam = fmaxf(normal_speed(P, wm, n), normal_speed(P, wp, n));
    atomicMax(&sL[e * 4 + f], __float_as_uint(lam));
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < kFaceIters; ++s) {
    const int it = tid + s * kThreads;
    if (it >= kTileE * S::NF) break;
    const int e = it / S::NF, fi = it - e * S::NF;
    const int f = fi / S::Nfp;
    float* row = sB + (3 * S::Np + fi) * S::NCOL + e * 5;
    if (e >= ne) {
#pragma unroll
      for (int v = 0; v < 5; ++v) row[v] = 0.0f;
      continue;
    }
    const float* sg = sS + e * 16 + f * 4;
    const float n[3] = {sg[0], sg[1], sg[2]};
    const float lam = __uint_as_float(sL[e * 4 + f]);
    Prim wm, wp;
    primitive(P, qm[s], wm);
    primitive(P, qp[s], wp);
    float fm[5], fp[5];
    normal_flux(P, wm, n, fm);
    normal_flux(P, wp, n, fp);
    const float hs = 0.5f * sg[3];
#pragma unroll
    for (int v = 0; v < 5; ++v) row[v] = hs * ((fm[v] - fp[v]) - lam * (qm[s][v] - qp[s][v]));
  }
  __syncthreads();

  // 4. contraction on MFMA: C[MP x NCOL] = A[MP x KT4] * B[KT4 x NCOL]
  const int wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lk = lane >> 4;
  const double dt = run ? run->dt : dt_host;
  for (int t = wave; t < S::MT * S::NT; t += kThreads / 64) {
    const int mt = t % S::MT, nt = t / S::MT;
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    const float* Ap = m.Aop + lk * S::MP + mt * 16 + lr;
    const float* Bp = sB + lk * S::NCOL + nt * 16 + lr;
#pragma unroll 4
    for (int ks = 0; ks < S::KT4 / 4; ++ks) {
      const float av = Ap[ks * 4 * S::MP];
      const float bv = Bp[ks * 4 * S::NCOL];
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
    }
    // 5. epilogue: lane holds rows mt*16 + 4*lk + r of column nt*16 + lr
    const int col = nt * 16 + lr;
    const int e = col / 5, v = col - e * 5;
    if (e < ne) {
      const int64_t base = (e0 + e) * S::ST + v * S::Np;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int node = mt * 16 + 4 * lk + r;
        if (node < S::Np) {
          const int64_t g = base + node;
          if (MODE == MODE_RHS) {
            out[g] = acc[r];
          } else {
            float rr = float(dt) * acc[r];
            if (a_rk != 0.0f) rr += a_rk * res[g];
            res[g] = rr;
            q_out[g] = sQ[e * S::ST + v * S::Np + node] + b_rk * rr;
          }
        }
      }
    }
  }
}

// ---- time step -------------------------------------------------------------

template <int N>
__global__ __launch_bounds__(256) void rate_kernel(DeviceMesh m, const float* __restrict__ q,
                                                   RunScalars* run) {
  using S = Shape<N>;
  const int64_t total = m.K * S::NF;
  float best = 0.0f;
  unsigned bad = 0u;
  for (int64_t it = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; it < total;
       it += int64_t(gridDim.x) * blockDim.x) {
    const int64_t k = it / S::NF;
    const int fi = int(it - k * S::NF);
    const int f = fi / S::Nfp, i = fi - f * S::Nfp;
    const int node = m.fmask[f * S::Nfp + i];
    float qq[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) qq[v] = q[k * S::ST + v * S::Np + node];
    Prim w;
    primitive(m.phys, qq, w);
    float speed2 = 0.0f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float u = m.phys.u0[d] + w.du[d];
      speed2 += u * u;
    }
    const float c = sqrtf(m.phys.gamma * w.p / w.rho);
    const float rate = m.phys.half_N1sq * float(m.sgeo[k * 16 + f * 4 + 3]) * (sqrtf(speed2) + c);
    if (!(w.rho > 0.0f) || !(w.p > 0.0f) || !(rate == rate)) bad = 1u;
    else best = fmaxf(best, rate);
  }
  // wavefront max, then one atomic per wave (order-independent)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    best = fmaxf(best, __shfl_xor(best, off));
    bad |= __shfl_xor(bad, off);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&run->rate_bits, __float_as_uint(best));
    if (bad) atomicOr(&run->bad, 1u);
  }
}

__global__ void finalize_kernel(RunScalars* run) {
  const float rate = __uint_as_float(run->rate_bits);
  run->dt = (rate > 0.0f) ? run->cfl / double(rate) : 0.0;
  if (run->bad && run->first_bad < 0) run->first_bad = run->step;
  run->rate_bits = 0u;
  run->bad = 0u;
}

__global__ void advance_kernel(RunScalars* run) {
  run->t += run->dt;
  run->step += 1;
}

// prim' (rho', u-u0, v-v0, w-w0, p') <-> q'
__global__ void prim_kernel(DeviceMesh m, const float* __restrict__ in, float* __restrict__ outp,
                            int inverse) {
  const int Np = m.Np;
  const int64_t total = m.K * Np;
  for (int64_t it = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; it < total;
       it += int64_t(gridDim.x) * blockDim.x) {
    const int64_t k = it / Np;
    const int i = int(it - k * Np);
    const int64_t base = k * 5 * Np + i;
    float x[5], y[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) x[v] = in[base + v * Np];
    if (!inverse) {
      const float du[3] = {x[1], x[2], x[3]};
      state_from(m.phys, x[0], du, x[4], y);
    } else {
      Prim w;
      primitive(m.phys, x, w);
      y[0] = w.rhop;
      y[1] = w.du[0];
      y[2] = w.du[1];
      y[3] = w.du[2];
      y[4] = w.pp;
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) outp[base + v * Np] = y[v];
  }
}

template <int N>
hipError_t stage_prepare() {
  using S = Shape<N>;
  const int lds = int(S::total * sizeof(float));
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&stage_kernel<N, MODE_RHS>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&stage_kernel<N, MODE_STAGE>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

template <int N>
hipError_t stage_dispatch(const DeviceMesh& m, int mode, const float* q_in, float* q_out,
                          float* res, float* out, float a, float b, double c, double t_host,
                          double dt_host, const RunScalars* run, hipStream_t s) {
  using S = Shape<N>;
  const int tiles = int((m.K + kTileE - 1) / kTileE);
  const size_t lds = size_t(S::total) * sizeof(float);
  if (mode == MODE_RHS)
    stage_kernel<N, MODE_RHS><<<tiles, kThreads, lds, s>>>(m, q_in, q_out, res, out, a, b, c,
                                                           t_host, dt_host, run);
  else
    stage_kernel<N, MODE_STAGE><<<tiles, kThreads, lds, s>>>(m, q_in, q_out, res, out, a, b, c,
                                                             t_host, dt_host, run);
  return hipGetLastError();
}

template <int N>
hipError_t rate_dispatch(const DeviceMesh& m, const float* q, RunScalars* run, hipStream_t s) {
  using S = Shape<N>;
  const int64_t total = m.K * S::NF;
  const int blocks = int(std::min<int64_t>((total + 255) / 256, 4096));
  rate_kernel<N><<<blocks, 256, 0, s>>>(m, q, run);
  return hipGetLastError();
}

}  // namespace

size_t stage_lds_bytes(int N) {
  switch (N) {
    case 1: return Shape<1>::total * sizeof(float);
    case 2: return Shape<2>::total * sizeof(float);
    case 3: return Shape<3>::total * sizeof(float);
    case 4: return Shape<4>::total * sizeof(float);
    case 5: return Shape<5>::total * sizeof(float);
    default: return 0;
  }
}

hipError_t prepare_kernels(int N) {
  switch (N) {
    case 1: return stage_prepare<1>();
    case 2: return stage_prepare<2>();
    case 3: return stage_prepare<3>();
    case 4: return stage_prepare<4>();
    case 5: return stage_prepare<5>();
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_stage(const DeviceMesh& m, int mode, const float* q_in, float* q_out, float* res,
                        float* out, float a, float b, double c, double t_host, double dt_host,
                        const RunScalars* run, hipStream_t s) {
  switch (m.N) {
    case 1: return stage_dispatch<1>(m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, s);
    case 2: return stage_dispatch<2>(m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, s);
    case 3: return stage_dispatch<3>(m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, s);
    case 4: return stage_dispatch<4>(m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, s);
    case 5: return stage_dispatch<5>(m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rate(const DeviceMesh& m, const float* q, RunScalars* run, hipStream_t s) {
  switch (m.N) {
    case 1: return rate_dispatch<1>(m, q, run, s);
    case 2: return rate_dispatch<2>(m, q, run, s);
    case 3: return rate_dispatch<3>(m, q, run, s);
    case 4: return rate_dispatch<4>(m, q, run, s);
    case 5: return rate_dispatch<5>(m, q, run, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_finalize(RunScalars* run, hipStream_t s) {
  finalize_kernel<<<1, 1, 0, s>>>(run);
  return hipGetLastError();
}

hipError_t launch_advance(RunScalars* run, hipStream_t s) {
  advance_kernel<<<1, 1, 0, s>>>(run);
  return hipGetLastError();
}

hipError_t launch_prim_to_state(const DeviceMesh& m, const float* prim, float* q, bool inverse,
                                hipStream_t s) {
  const int64_t total = m.K * m.Np;
  const int blocks = int(std::min<int64_t>((total + 255) / 256, 8192));
  prim_kernel<<<blocks, 256, 0, s>>>(m, prim, q, inverse ? 1 : 0);
  return hipGetLastError();
}

}  // namespace dg
