// Weak-form right-hand side with Gauss quadrature (gfx950), N = 1, 2.
//
// Appendix A's Galerkin statement, integrated with quadrature rather than
// by nodal interpolation of the flux:
//   M_K dq/dt = int_K grad(l_i) . F(q) dx - oint_dK l_i F* . n ds,
// volume points exact to degree 2N, face points to degree 2N + 1, q the
// nodal values of the order-N nodes (the same polynomial space and state
// layout as the nodal scheme); the face rule is symmetric under the face's
// vertex permutations, so both sides of a face integrate at the same points
// and the scheme conserves.  Four lanes per element: each holds the
// element's nodal values and its own right-hand-side accumulators in
// registers, takes every fourth volume point and one face, and the four
// partial sums are added by lane shuffles (the same order in every lane, so
// all four hold bit-identical sums); the per-order tables
// (interpolation to the volume and face points, the weighted derivative
// and lifting operators, and the neighbour-side interpolation for every
// face pairing and orientation) are staged in LDS and read at addresses
// that are the same for every lane, except the neighbour table.  F* is the
// local Lax-Friedrichs flux with one speed per face (largest |u.n| + c over
// the face's points and both sides); fluxes are perturbations from the
// ambient state (its constant flux integrates to zero).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "physics.hpp"
#include "quad.hpp"

namespace dg {
namespace {

template <int N>
struct QShape {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
  static constexpr int Nq = (N + 1) * (N + 1) * (N + 1);
  static constexpr int Nfq = 7;  // Radon's symmetric face rule
  static constexpr int ST = 5 * Np;
  static constexpr int oBv = 0;
  static constexpr int oDw = oBv + Nq * Np;
  static constexpr int oBf = oDw + 3 * Np * Nq;
  static constexpr int oLq = oBf + 4 * Nfq * Np;
  static constexpr int oBnb = oLq + 4 * Np * Nfq;
  static constexpr int total = oBnb + 96 * Nfq * Np;
};

// An element's ST contiguous floats with the widest vector accesses its
// alignment allows (element blocks of 80 B at N = 1, 200 B at N = 2).
template <int ST>
struct ElemIO {
  static constexpr int W = (ST * 4) % 16 == 0 ? 4 : ((ST * 4) % 8 == 0 ? 2 : 1);
  __device__ static __forceinline__ void load(const float* p, float (&x)[ST]) {
#pragma unroll
    for (int j = 0; j < ST / W; ++j) {
      if constexpr (W == 4) {
        const float4 v = reinterpret_cast<const float4*>(p)[j];
        x[4 * j] = v.x; x[4 * j + 1] = v.y; x[4 * j + 2] = v.z; x[4 * j + 3] = v.w;
      } else if constexpr (W == 2) {
        const float2 v = reinterpret_cast<const float2*>(p)[j];
        x[2 * j] = v.x; x[2 * j + 1] = v.y;
      } else {
        x[j] = p[j];
      }
    }
  }
  __device__ static __forceinline__ void store(float* p, const float (&x)[ST]) {
#pragma unroll
    for (int j = 0; j < ST / W; ++j) {
      if constexpr (W == 4) {
        reinterpret_cast<float4*>(p)[j] = make_float4(x[4 * j], x[4 * j + 1], x[4 * j + 2], x[4 * j + 3]);
      } else if constexpr (W == 2) {
        reinterpret_cast<float2*>(p)[j] = make_float2(x[2 * j], x[2 * j + 1]);
      } else {
        p[j] = x[j];
      }
    }
  }
};

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
__global__ __launch_bounds__(256) void quad_kernel(DeviceMesh m, const float* __restrict__ tab,
                                                   const float* __restrict__ q_in,
                                                   const float* q_base, float* q_out,
                                                   float* __restrict__ out, float alpha,
                                                   float beta, double c_rk, double t_host,
                                                   double dt_host, RunScalars* run,
                                                   int rate_out) {
  using S = QShape<N>;
  constexpr int Np = S::Np, Nfp = S::Nfp, Nq = S::Nq, Nfq = S::Nfq, ST = S::ST;
  extern __shared__ float T[];
  for (int i = threadIdx.x; i < S::total; i += blockDim.x) T[i] = tab[i];
  __syncthreads();
  const Phys& P = m.phys;
  const double tst = stage_time(c_rk, t_host, dt_host, run);
  const float pin = inflow_pressure(P, tst);
  const float dt = float(run ? run->dt : dt_host);
  float rate_best = 0.0f;
  unsigned rate_bad = 0u;

  constexpr int kLanes = 4;          // lanes per element (adjacent lanes)
  const int g = threadIdx.x & (kLanes - 1);
  for (int64_t k = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kLanes; k < m.K;
       k += int64_t(gridDim.x) * blockDim.x / kLanes) {
    float qe[5][Np], acc[5][Np];
    {
      float flat[ST];
      ElemIO<ST>::load(q_in + k * ST, flat);
#pragma unroll
      for (int v = 0; v < 5; ++v)
#pragma unroll
        for (int i = 0; i < Np; ++i) {
          qe[v][i] = flat[v * Np + i];
          acc[v][i] = 0.0f;
        }
    }
    float G[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) G[i] = float(m.vgeo[k * 9 + i]);

    // volume: sum_q w_q sum_a (d l_i / d r_a) Fc_a, with M^-1 folded in
#pragma unroll 1
    for (int q = g; q < Nq; q += kLanes) {
      float u[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        float x = 0.0f;
#pragma unroll
        for (int i = 0; i < Np; ++i) x += T[S::oBv + q * Np + i] * qe[v][i];
        u[v] = x;
      }
      Prim w;
      primitive<true>(P, u, w);
      float F[3][5];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const float d[3] = {G[a * 3], G[a * 3 + 1], G[a * 3 + 2]};
        normal_flux<true>(P, w, d, F[a]);
      }
#pragma unroll
      for (int i = 0; i < Np; ++i) {
        const float d0 = T[S::oDw + (0 * Np + i) * Nq + q];
        const float d1 = T[S::oDw + (1 * Np + i) * Nq + q];
        const float d2 = T[S::oDw + (2 * Np + i) * Nq + q];
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[v][i] += d0 * F[0][v] + d1 * F[1][v] + d2 * F[2][v];
      }
    }

    // faces: - Fscale_f sum_qf M^-1 l_i w F*.n
    {
      const int f = g;  // this lane's face
      const int nb = m.nbr[k * 4 + f];
      const float n[3] = {float(m.sgeo[k * 16 + f * 4]), float(m.sgeo[k * 16 + f * 4 + 1]),
                          float(m.sgeo[k * 16 + f * 4 + 2])};
      const float fs = float(m.sgeo[k * 16 + f * 4 + 3]);
      float qn[5][Np];
      const float* Bn = T;
      if (nb >= 0) {
        float flat[ST];
        ElemIO<ST>::load(q_in + int64_t(nb) * ST, flat);
#pragma unroll
        for (int v = 0; v < 5; ++v)
#pragma unroll
          for (int i = 0; i < Np; ++i) qn[v][i] = flat[v * Np + i];
        const int fi = m.finfo[k * 4 + f];
        Bn = T + S::oBnb + ((f * 4 + (fi & 3)) * 6 + (fi >> 2)) * Nfq * Np;
      } else {
#pragma unroll
        for (int v = 0; v < 5; ++v)
#pragma unroll
          for (int i = 0; i < Np; ++i) qn[v][i] = 0.0f;
      }
      const int tag = nb >= 0 ? 0 : ((-nb) & 7);
      auto sides = [&](int qf, float (&qm)[5], Prim& wm, float (&qp)[5], Prim& wp)
          __attribute__((always_inline)) {
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          float x = 0.0f, y = 0.0f;
#pragma unroll
          for (int i = 0; i < Np; ++i) {
            x += T[S::oBf + (f * Nfq + qf) * Np + i] * qe[v][i];
            y += Bn[qf * Np + i] * qn[v][i];
          }
          qm[v] = x;
          qp[v] = y;
        }
        primitive<true>(P, qm, wm);
        if (nb < 0) ghost(P, tag, qm, wm, n, pin, qp);
        primitive<true>(P, qp, wp);
      };
      if constexpr (N == 1) {
        // one pass over the face's points: lambda is one per face, so its
        // term lambda (q- - q+)/2 is lifted separately and scaled at the end
        float lam = 0.0f;
        float dql[5][Np];
#pragma unroll
        for (int v = 0; v < 5; ++v)
#pragma unroll
          for (int i = 0; i < Np; ++i) dql[v][i] = 0.0f;
#pragma unroll 1
        for (int qf = 0; qf < Nfq; ++qf) {
          float qm[5], qp[5], fm[5], fp[5];
          Prim wm, wp;
          sides(qf, qm, wm, qp, wp);
          lam = fmaxf(lam, fmaxf(normal_speed<true>(P, wm, n), normal_speed<true>(P, wp, n)));
          normal_flux<true>(P, wm, n, fm);
          normal_flux<true>(P, wp, n, fp);
          float Fa[5], dq[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            Fa[v] = 0.5f * fs * (fm[v] + fp[v]);
            dq[v] = qm[v] - qp[v];
          }
#pragma unroll
          for (int i = 0; i < Np; ++i) {
            const float l = T[S::oLq + (f * Np + i) * Nfq + qf];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
              acc[v][i] -= l * Fa[v];
              dql[v][i] += l * dq[v];
            }
          }
        }
        const float cl = 0.5f * fs * lam;
#pragma unroll
        for (int v = 0; v < 5; ++v)
#pragma unroll
          for (int i = 0; i < Np; ++i) acc[v][i] -= cl * dql[v][i];
      } else {  // at N = 2 the extra accumulators would cost occupancy: two passes
        float lam = 0.0f;
#pragma unroll 1
        for (int qf = 0; qf < Nfq; ++qf) {
          float qm[5], qp[5];
          Prim wm, wp;
          sides(qf, qm, wm, qp, wp);
          lam = fmaxf(lam, fmaxf(normal_speed<true>(P, wm, n), normal_speed<true>(P, wp, n)));
        }
#pragma unroll 1
        for (int qf = 0; qf < Nfq; ++qf) {
          float qm[5], qp[5], fm[5], fp[5];
          Prim wm, wp;
          sides(qf, qm, wm, qp, wp);
          normal_flux<true>(P, wm, n, fm);
          normal_flux<true>(P, wp, n, fp);
          float Fn[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) Fn[v] = fs * (0.5f * (fm[v] + fp[v]) + 0.5f * lam * (qm[v] - qp[v]));
#pragma unroll
          for (int i = 0; i < Np; ++i) {
            const float l = T[S::oLq + (f * Np + i) * Nfq + qf];
#pragma unroll
            for (int v = 0; v < 5; ++v) acc[v][i] -= l * Fn[v];
          }
        }
      }
    }

    // the four lanes' partial sums
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int i = 0; i < Np; ++i) {
        acc[v][i] += __shfl_xor(acc[v][i], 1);
        acc[v][i] += __shfl_xor(acc[v][i], 2);
      }

    // epilogue (stores by the element's first lane)
    if (MODE == MODE_RHS) {
      float flat[ST];
#pragma unroll
      for (int v = 0; v < 5; ++v)
#pragma unroll
        for (int i = 0; i < Np; ++i) flat[v * Np + i] = acc[v][i];
      if (g == 0) ElemIO<ST>::store(out + k * ST, flat);
    } else {
      float flat[ST];
      if (alpha != 0.0f) {
        ElemIO<ST>::load(q_base + k * ST, flat);
      } else {
#pragma unroll
        for (int j = 0; j < ST; ++j) flat[j] = 0.0f;
      }
#pragma unroll
      for (int v = 0; v < 5; ++v)
#pragma unroll
        for (int i = 0; i < Np; ++i) {
          const float qn_ = alpha * flat[v * Np + i] + beta * (qe[v][i] + dt * acc[v][i]);
          flat[v * Np + i] = qn_;
          qe[v][i] = qn_;
        }
      if (g == 0) ElemIO<ST>::store(q_out + k * ST, flat);
      if (rate_out) {  // next step's CFL rate from the new state's nodes on this lane's face
        {
          const int f = g;
          const float fs = float(m.sgeo[k * 16 + f * 4 + 3]);
#pragma unroll 1
          for (int ii = 0; ii < Nfp; ++ii) {
            const int node = m.fmask[f * Nfp + ii];
            float qq[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
              float x = 0.0f;
#pragma unroll
              for (int i = 0; i < Np; ++i) x = (i == node) ? qe[v][i] : x;
              qq[v] = x;
            }
            Prim w;
            primitive<true>(P, qq, w);
            float u2 = 0.0f;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              const float uu = P.u0[d] + w.du[d];
              u2 += uu * uu;
            }
            const float rate = P.half_N1sq * fs * (sqrtf(u2) + sqrtf(P.gamma * w.p / w.rho));
            if (!(w.rho > 0.0f) || !(w.p > 0.0f) || !(rate == rate)) rate_bad = 1u;
            else rate_best = fmaxf(rate_best, rate);
          }
        }
      }
    }
  }
  if (MODE == MODE_STAGE && rate_out) {  // wavefront, then block, then one atomic per block
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      rate_best = fmaxf(rate_best, __shfl_xor(rate_best, off));
      rate_bad |= __shfl_xor(rate_bad, off);
    }
    __shared__ float wbest[4];
    __shared__ unsigned wbad[4];
    if ((threadIdx.x & 63) == 0) {
      wbest[threadIdx.x >> 6] = rate_best;
      wbad[threadIdx.x >> 6] = rate_bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const float b = fmaxf(fmaxf(wbest[0], wbest[1]), fmaxf(wbest[2], wbest[3]));
      atomicMax(&run->rate_bits, __float_as_uint(b));
      if (wbad[0] | wbad[1] | wbad[2] | wbad[3]) atomicOr(&run->bad, 1u);
    }
  }
}

template <int N, int MODE>
hipError_t launch_nm(const DeviceMesh& m, const float* q_in, const float* q_base, float* q_out,
                     float* out, float alpha, float beta, double c, double t_host, double dt_host,
                     RunScalars* run, int rate_out, hipStream_t s) {
  const size_t lds = size_t(QShape<N>::total) * sizeof(float);
  const void* fn = reinterpret_cast<const void*>(&quad_kernel<N, MODE>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (e != hipSuccess) return e;
  const int64_t want = (4 * m.K + 255) / 256;   // four lanes per element
  const int blocks = int(std::max<int64_t>(1, std::min<int64_t>(want, int64_t(m.num_cu) * 16)));
  quad_kernel<N, MODE><<<blocks, 256, lds, s>>>(m, m.qtab, q_in, q_base, q_out, out, alpha, beta,
                                                c, t_host, dt_host, run, rate_out);
  return hipGetLastError();
}

}  // namespace

size_t quad_table_floats(int N) {
  switch (N) {
    case 1: return QShape<1>::total;
    case 2: return QShape<2>::total;
    default: return 0;
  }
}

hipError_t launch_quad(const DeviceMesh& m, int mode, const float* q_in, const float* q_base,
                       float* q_out, float* out, float alpha, float beta, double c,
                       double t_host, double dt_host, RunScalars* run, int rate_out,
                       hipStream_t s) {
  const int ro = (run != nullptr && rate_out) ? 1 : 0;
  if (m.N == 1)
    return mode == MODE_RHS
               ? launch_nm<1, MODE_RHS>(m, q_in, q_base, q_out, out, alpha, beta, c, t_host, dt_host, run, 0, s)
               : launch_nm<1, MODE_STAGE>(m, q_in, q_base, q_out, out, alpha, beta, c, t_host, dt_host, run, ro, s);
  if (m.N == 2)
    return mode == MODE_RHS
               ? launch_nm<2, MODE_RHS>(m, q_in, q_base, q_out, out, alpha, beta, c, t_host, dt_host, run, 0, s)
               : launch_nm<2, MODE_STAGE>(m, q_in, q_base, q_out, out, alpha, beta, c, t_host, dt_host, run, ro, s);
  return hipErrorInvalidValue;
}

}  // namespace dg
