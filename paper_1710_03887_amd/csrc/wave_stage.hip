// Wavefront-private fused stage kernel (gfx950 / CDNA4).
//
// Same arithmetic as the tile-cooperative stage kernel, organized so that no
// wavefront ever waits for another: a wavefront owns a tile of 16 elements
// (the 16 MFMA columns) from its loads to its stores.  One block of eight
// wavefronts per CU shares the LDS-resident operator A = [-Dr -Ds -Dt | LIFT]
// (Appendix A, Eq. 10); each wavefront has a private LDS slot for its tile's
// state q' [16][5][Np] and FP64 geometry, filled by asynchronous
// global->LDS copies, and holds the exterior traces of its tile in registers
// (gathered once per tile).  Per tile:
//   1. the local Lax-Friedrichs speed of every element face, max over its
//      nodes and both sides of |u.n| + c, reduced across the four lane groups
//      with shuffles;
//   2. volume: contravariant fluxes of each node quad straight into MFMA f32
//      16x16x4 products against the operator's derivative rows;
//   3. surface: the jump Fscale/2 [n.(F- - F+) - lambda (q- - q+)] of each
//      face-node quad against the LIFT rows;
//   4. the fused low-storage RK update (or the right-hand side) from the
//      accumulators, and on the last stage of a step the next time-step rate.
// With no block barriers in the loop, the two wavefronts of a SIMD overlap
// one another's memory waits, VALU work and MFMA work freely.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"

namespace dg {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void* lds_ptr_t;

constexpr int kWW = 8;   // wavefronts per block, one block per CU
constexpr int kTE = 16;  // elements per tile (MFMA n)

template <int N>
struct WShape {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
  static constexpr int NF = 4 * Nfp;
  static constexpr int NFQ = NF / 4;
  static constexpr int NNQ = (Np + 3) / 4;
  static constexpr int NQP = 4 * NNQ;
  static constexpr int KV = 3 * NQP;
  static constexpr int KT = KV + NF;
  static constexpr int MP = (Np + 15) / 16 * 16;
  static constexpr int MT = MP / 16;
  static constexpr int AS = (MP % 32 == 16) ? MP : MP + 16;
  static constexpr int ST = 5 * Np;
  // LDS in floats: operator | byte tables | per wavefront: state, FP64 geometry
  static constexpr int tabBytes = NF + 96 * Nfp + Np;
  static constexpr int oTab = KT * AS;
  static constexpr int oWave = oTab + (tabBytes + 15) / 16 * 4;
  static constexpr int geoFloats = kTE * 25 * 2;  // [16][9] + [16][16] doubles
  static constexpr int waveFloats = kTE * ST + geoFloats + kTE * 4;  // + FP32 Fscale
  static_assert(kTE * MP <= geoFloats, "transpose scratch fits over the geometry");
  static constexpr int total = oWave + kWW * waveFloats;
  static_assert((kTE * ST) % 4 == 0, "state tile is whole 16-byte chunks");
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

template <class T>
__device__ __forceinline__ T pick4(const T* x, int f) {
  return f == 0 ? x[0] : f == 1 ? x[1] : f == 2 ? x[2] : x[3];
}

// An empty asm that the compiler must assume changes x: the surface pass
// recomputes the traces' primitive states instead of keeping every one of
// them alive from the speed pass (which would not fit in registers).
__device__ __forceinline__ float opaque(float x) {
  asm volatile("" : "+v"(x));
  return x;
}

__device__ __forceinline__ floatx4 mfma(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// wait until every LDS access of this wavefront has completed (before an
// asynchronous copy overwrites its slot); vmcnt and expcnt are left open
__device__ __forceinline__ void wait_lds() { __builtin_amdgcn_s_waitcnt(0xc07f); }

// Hand-off of LDS data between the lanes of one wavefront.  The hardware
// performs a wavefront's LDS accesses in program order, but the compiler
// reasons per lane: without a convergent point it may, for example, let lanes
// that skip a read loop run the following stores first.  The fences order
// the memory operations at wavefront scope (no instruction on gfx950), the
// wave barrier keeps all lanes together at this point.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int N, int MODE, bool MOVING>
__global__ __launch_bounds__(64 * kWW) __attribute__((amdgpu_waves_per_eu(2)))
void wave_stage_kernel(DeviceMesh m, const float* __restrict__ q_in, float* __restrict__ q_out,
                       float* __restrict__ res, float* __restrict__ out, float a_rk, float b_rk,
                       double c_rk, double t_host, double dt_host, RunScalars* run,
                       int rate_out) {
  using S = WShape<N>;
  constexpr int Np = S::Np, Nfp = S::Nfp, ST = S::ST, MT = S::MT, AS = S::AS, NFQ = S::NFQ;
  extern __shared__ float lds[];
  const float* sA = lds;
  uint8_t* sFm = reinterpret_cast<uint8_t*>(lds + S::oTab);
  uint8_t* sNN = sFm + S::NF;
  uint8_t* sNF = sNN + 96 * Nfp;
  const Phys& P = m.phys;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int e = lane & 15, g = lane >> 4;
  float* sQ = lds + S::oWave + w * S::waveFloats;
  const double* sV = reinterpret_cast<const double*>(sQ + kTE * ST);  // [16][9]
  const double* sS = sV + kTE * 9;                                    // [16][16]
  float* sFsc = sQ + kTE * ST + S::geoFloats;                         // [16][4] Fscale

  for (int i = tid; i < S::KT * AS; i += 64 * kWW) lds[i] = m.Aop[i];
  for (int i = tid; i < S::NF; i += 64 * kWW) sFm[i] = m.fmask[i];
  for (int i = tid; i < 96 * Nfp; i += 64 * kWW) sNN[i] = m.nbr_node[i];
  for (int i = tid; i < Np; i += 64 * kWW) {
    int mask = 0;
    for (int f = 0; f < 4; ++f)
      for (int ii = 0; ii < Nfp; ++ii)
        if (m.fmask[f * Nfp + ii] == i) mask |= 1 << f;
    sNF[i] = uint8_t(mask);
  }
  __syncthreads();  // the only block barrier

  const double tst = stage_time(c_rk, t_host, dt_host, run);
  const float pin = inflow_pressure(P, tst);
  const float dt = float(run ? run->dt : dt_host);

  const int64_t ntiles = (m.K + kTE - 1) / kTE;
  const int G = gridDim.x, nX = G < 8 ? G : 8;
  const int x = blockIdx.x % nX, jb = blockIdx.x / nX;
  const int Gx = G / nX + (x < G % nX ? 1 : 0);
  const int64_t c0 = ntiles * x / nX, c1 = ntiles * (x + 1) / nX;
  const int64_t stride = int64_t(Gx) * kWW;

  // connectivity of the lane's element, one tile ahead
  auto load_conn = [&](int64_t t, int4& nb4, unsigned& fi4) {
    const int64_t kk = t * kTE + e;
    if (t < c1 && kk < m.K) {
      nb4 = reinterpret_cast<const int4*>(m.nbr)[kk];
      fi4 = reinterpret_cast<const unsigned*>(m.finfo)[kk];
    } else {
      nb4 = make_int4(-BC_PASSTHRU, -BC_PASSTHRU, -BC_PASSTHRU, -BC_PASSTHRU);
      fi4 = 0u;
    }
  };
  int4 nbN;
  unsigned fiN;
  load_conn(c0 + int64_t(jb) * kWW + w, nbN, fiN);

  float rate_best = 0.0f;
  unsigned rate_bad = 0u;
  for (int64_t tile = c0 + int64_t(jb) * kWW + w; tile < c1; tile += stride) {
    // lane coordinates re-derived every tile through an opaque copy, so that
    // the many lane-dependent LDS addresses are not hoisted out of the loop
    // (each would hold a register across all tiles)
    int lane_t = lane;
    asm volatile("" : "+v"(lane_t));
    const int e = lane_t & 15, g = lane_t >> 4;
    const int64_t k0 = tile * kTE;
    const int ne = int(min<int64_t>(kTE, m.K - k0));
    const bool valid = e < ne;
    const int nbr[4] = {nbN.x, nbN.y, nbN.z, nbN.w};
    const unsigned fi4 = fiN;

    // A. loads: own state and FP64 geometry into this wavefront's LDS slot
    // (asynchronous), exterior traces into registers
    wave_sync();  // every lane is done with the previous tile's slot
    wait_lds();
    if (ne == kTE) {
      constexpr int n4 = kTE * ST / 4;
      const float* qg = q_in + k0 * ST;
#pragma unroll
      for (int j = 0; j < (n4 + 63) / 64; ++j) {
        const int i4 = j * 64 + lane;
        if (i4 < n4)
          __builtin_amdgcn_global_load_lds((void*)(qg + 4 * i4), (lds_ptr_t)(sQ + j * 256), 16, 0, 0);
      }
      const char* vsrc = reinterpret_cast<const char*>(m.vgeo + k0 * 9);
      const char* ssrc = reinterpret_cast<const char*>(m.sgeo + k0 * 16);
      char* gdst = reinterpret_cast<char*>(sQ + kTE * ST);
      __builtin_amdgcn_global_load_lds((void*)(vsrc + 16 * lane), (lds_ptr_t)(gdst), 16, 0, 0);
      if (lane < 8)
        __builtin_amdgcn_global_load_lds((void*)(vsrc + 1024 + 16 * lane), (lds_ptr_t)(gdst + 1024),
                                         16, 0, 0);
      __builtin_amdgcn_global_load_lds((void*)(ssrc + 16 * lane), (lds_ptr_t)(gdst + 1152), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((void*)(ssrc + 1024 + 16 * lane), (lds_ptr_t)(gdst + 2176),
                                       16, 0, 0);
    } else {
      for (int i = lane; i < kTE * ST; i += 64) sQ[i] = i < ne * ST ? q_in[k0 * ST + i] : 0.0f;
      double* gd = reinterpret_cast<double*>(sQ + kTE * ST);
      for (int i = lane; i < kTE * 9; i += 64) gd[i] = i < ne * 9 ? m.vgeo[k0 * 9 + i] : 0.0;
      for (int i = lane; i < kTE * 16; i += 64)
        gd[kTE * 9 + i] = i < ne * 16 ? m.sgeo[k0 * 16 + i] : 0.0;
    }
    load_conn(tile + stride, nbN, fiN);

    // exterior traces of face f, lane (e, g) taking face nodes 4q + g (the
    // last quad padded); branch-free: lanes with no stored exterior trace
    // load from their own element and discard the value
    constexpr int QF = (Nfp + 3) / 4;
    const float* self = q_in + (k0 + (valid ? e : 0)) * ST;
    auto gather = [&](int f, float (&t)[QF][5]) __attribute__((always_inline)) {
      const int nb = nbr[f];
      const int inf = nb >= 0 ? (fi4 >> (8 * f)) & 0xff : 0;  // meaningful on interior faces only
      const bool inner = valid && nb >= 0;
      const bool learned = valid && nb < 0 && m.lghost && ((-nb) & 7) == BC_LEARNED;
#pragma unroll
      for (int q = 0; q < QF; ++q) {
        const int ii = min(4 * q + g, Nfp - 1);
        const int n2 = sNN[((f * 4 + (inf & 3)) * 6 + (inf >> 2)) * Nfp + ii];
        const float* src = inner ? q_in + int64_t(nb) * ST + n2
                                 : learned ? m.lghost + int64_t((-nb) >> 3) * ST + ii : self;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          const float val = src[v * Np];
          t[q][v] = (inner || learned) ? val : 0.0f;
        }
      }
    };
    float trn[QF][5];
    gather(0, trn);
    __builtin_amdgcn_s_waitcnt(0);  // state, geometry and face-0 traces have landed
    wave_sync();

    // geometry of the lane's element in FP32
    float gm[9], nx[4], ny[4], nz[4], fs[4];
#pragma unroll
    for (int i = 0; i < 9; ++i) gm[i] = float(sV[e * 9 + i]);
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      nx[f] = float(sS[e * 16 + f * 4 + 0]);
      ny[f] = float(sS[e * 16 + f * 4 + 1]);
      nz[f] = float(sS[e * 16 + f * 4 + 2]);
      fs[f] = float(sS[e * 16 + f * 4 + 3]);
    }
    const bool lrn = m.lghost != nullptr;

    floatx4 acc[5][MT];
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[v][mt] = floatx4{0.f, 0.f, 0.f, 0.f};

    // 1. volume
#pragma unroll
    for (int nq = 0; nq < S::NNQ; ++nq) {
      const int j = 4 * nq + g;
      float F[3][5];
      if (j < Np && valid) {
        float q[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) q[v] = sQ[e * ST + v * Np + j];
        Prim wv;
        primitive<MOVING>(P, q, wv);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float d[3] = {gm[a * 3 + 0], gm[a * 3 + 1], gm[a * 3 + 2]};
          normal_flux<MOVING>(P, wv, d, F[a]);
        }
      } else {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int v = 0; v < 5; ++v) F[a][v] = 0.0f;
      }
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const float av = sA[(a * S::NQP + j) * AS + mt * 16 + e];
#pragma unroll
          for (int v = 0; v < 5; ++v) acc[v][mt] = mfma(av, F[a][v], acc[v][mt]);
        }
    }

    // 2. faces one at a time (the next face's traces in flight meanwhile):
    //    the face's Lax-Friedrichs speed, max over its nodes and both sides
    //    of |u.n| + c, then the jump Fscale/2 [n.(F- - F+) - lambda (q- - q+)]
    //    against the LIFT rows
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      float trc[QF][5];
#pragma unroll
      for (int q = 0; q < QF; ++q)
#pragma unroll
        for (int v = 0; v < 5; ++v) trc[q][v] = trn[q][v];
      if (f < 3) gather(f + 1, trn);
      const float n[3] = {nx[f], ny[f], nz[f]};
      const int nb = valid ? nbr[f] : -BC_PASSTHRU;
      const bool stored = nb >= 0 || (lrn && ((-nb) & 7) == BC_LEARNED);
      float dfl[QF][5], dql[QF][5];
      float lam = 0.0f;
#pragma unroll
      for (int q = 0; q < QF; ++q) {
        const int ii = 4 * q + g;
        const int node = sFm[f * Nfp + min(ii, Nfp - 1)];
        float qm[5], qp[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) qm[v] = sQ[e * ST + v * Np + node];
        Prim wm;
        primitive<MOVING>(P, qm, wm);
        if (stored) {
#pragma unroll
          for (int v = 0; v < 5; ++v) qp[v] = trc[q][v];
        } else {
          ghost(P, -nb, qm, wm, n, pin, qp);
        }
        Prim wp;
        primitive<MOVING>(P, qp, wp);
        const float sp = fmaxf(normal_speed<MOVING>(P, wm, n), normal_speed<MOVING>(P, wp, n));
        if (ii < Nfp) lam = fmaxf(lam, sp);
        float fm[5], fp[5];
        normal_flux<MOVING>(P, wm, n, fm);
        normal_flux<MOVING>(P, wp, n, fp);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          dfl[q][v] = fm[v] - fp[v];
          dql[q][v] = qm[v] - qp[v];
        }
      }
      lam = fmaxf(lam, __shfl_xor(lam, 16));
      lam = fmaxf(lam, __shfl_xor(lam, 32));
      const float hs = valid ? 0.5f * fs[f] : 0.0f;
#pragma unroll
      for (int q = 0; q < QF; ++q) {
        const int ii = 4 * q + g;
        const float h = ii < Nfp ? hs : 0.0f;
        float dF[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) dF[v] = h * (dfl[q][v] - lam * dql[q][v]);
        const int row = S::KV + f * Nfp + min(ii, Nfp - 1);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const float av = sA[row * AS + mt * 16 + e];
#pragma unroll
          for (int v = 0; v < 5; ++v) acc[v][mt] = mfma(av, dF[v], acc[v][mt]);
        }
      }
    }

    // 4. epilogue, one variable at a time: the accumulators (lane (g, e)
    // holds nodes mt*16 + 4g + r of element e) are transposed through the
    // slot's geometry area so that residual and state are read and written
    // with element-contiguous runs
    float* sT = sQ + kTE * ST;  // [16][MP], the FP64 geometry is in registers by now
#pragma unroll
    for (int v = 0; v < 5; ++v) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
        *reinterpret_cast<floatx4*>(sT + e * S::MP + mt * 16 + 4 * g) = acc[v][mt];
      wave_sync();
      for (int idx = lane; idx < ne * Np; idx += 64) {
        const int el = idx / Np, node = idx - el * Np;
        const float a = sT[el * S::MP + node];
        const int64_t gx = (k0 + el) * ST + v * Np + node;
        if (MODE == MODE_RHS) {
          out[gx] = a;
        } else {
          const float rr = dt * a + (a_rk != 0.0f ? a_rk * res[gx] : 0.0f);
          res[gx] = rr;
          const float qn = sQ[el * ST + v * Np + node] + b_rk * rr;
          q_out[gx] = qn;
          if (rate_out) sQ[el * ST + v * Np + node] = qn;
        }
      }
      wave_sync();  // the transpose slot is read before the next variable's stores
    }
    // time-step rule for the next step from the new state (last stage only)
    if (MODE == MODE_STAGE && rate_out) {
#pragma unroll
      for (int f = 0; f < 4; ++f) sFsc[e * 4 + f] = fs[f];
      wave_sync();
      for (int idx = lane; idx < ne * S::NF; idx += 64) {
        const int el = idx / S::NF, i = idx - el * S::NF, f = i / Nfp;
        const int node = sFm[i];
        float qq[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) qq[v] = sQ[el * ST + v * Np + node];
        Prim wq;
        primitive<MOVING>(P, qq, wq);
        float u2 = 0.0f;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const float u = P.u0[d] + wq.du[d];
          u2 += u * u;
        }
        const float rate = P.half_N1sq * sFsc[el * 4 + f] * (sqrtf(u2) + sqrtf(P.gamma * wq.p / wq.rho));
        if (!(wq.rho > 0.0f) || !(wq.p > 0.0f) || !(rate == rate)) rate_bad = 1u;
        else rate_best = fmaxf(rate_best, rate);
      }
    }
  }

  if (MODE == MODE_STAGE && rate_out) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      rate_best = fmaxf(rate_best, __shfl_xor(rate_best, off));
      rate_bad |= __shfl_xor(rate_bad, off);
    }
    if (lane == 0) {
      atomicMax(&run->rate_bits, __float_as_uint(rate_best));
      if (rate_bad) atomicOr(&run->bad, 1u);
    }
  }
}

template <int N, int MODE, bool MOVING>
hipError_t launch_nm(const DeviceMesh& m, const float* q_in, float* q_out, float* res, float* out,
                     float a, float b, double c, double t_host, double dt_host, RunScalars* run,
                     int rate_out, hipStream_t s) {
  const size_t lds = size_t(WShape<N>::total) * sizeof(float);
  const void* fn = reinterpret_cast<const void*>(&wave_stage_kernel<N, MODE, MOVING>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (e != hipSuccess) return e;
  const int64_t tiles = (m.K + kTE - 1) / kTE;
  const int blocks = int(std::max<int64_t>(1, std::min<int64_t>((tiles + kWW - 1) / kWW, m.num_cu)));
  wave_stage_kernel<N, MODE, MOVING><<<blocks, 64 * kWW, lds, s>>>(m, q_in, q_out, res, out, a, b,
                                                                    c, t_host, dt_host, run,
                                                                    rate_out);
  return hipGetLastError();
}

template <int N>
hipError_t launch_n(const DeviceMesh& m, int mode, const float* q_in, float* q_out, float* res,
                    float* out, float a, float b, double c, double t_host, double dt_host,
                    RunScalars* run, int rate_out, hipStream_t s) {
  const bool moving = m.phys.u0[0] != 0.0f || m.phys.u0[1] != 0.0f || m.phys.u0[2] != 0.0f;
  if (mode == MODE_RHS)
    return moving ? launch_nm<N, MODE_RHS, true>(m, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, 0, s)
                  : launch_nm<N, MODE_RHS, false>(m, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, 0, s);
  return moving ? launch_nm<N, MODE_STAGE, true>(m, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, rate_out, s)
                : launch_nm<N, MODE_STAGE, false>(m, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, rate_out, s);
}

}  // namespace

bool wave_stage_supported(int N, int precision) { return precision == 0 && N >= 1 && N <= 4; }

hipError_t launch_wave_stage(const DeviceMesh& m, int mode, const float* q_in, float* q_out,
                             float* res, float* out, float a, float b, double c, double t_host,
                             double dt_host, RunScalars* run, int rate_out, hipStream_t s) {
  const int ro = (run != nullptr && rate_out) ? 1 : 0;
  switch (m.N) {
    case 1: return launch_n<1>(m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, ro, s);
    case 2: return launch_n<2>(m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, ro, s);
    case 3: return launch_n<3>(m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, ro, s);
    case 4: return launch_n<4>(m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, ro, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dg
