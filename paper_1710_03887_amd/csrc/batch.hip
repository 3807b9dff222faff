// Batched-ensemble stage kernel (gfx950).
//
// A wavefront owns one element of one geometry and all 16 members of the
// ensemble: the 16 MFMA columns are the members, so every state access
// q[k][v][node][0..15] and every neighbour gather is one coalesced 64-byte
// run, and the element's geometry and connectivity are read once for 16
// solves.  The per-element work is the same as in the single-solve kernel:
// Lax-Friedrichs speeds per face and member (reduced with wavefront
// shuffles), contravariant volume fluxes and surface jumps fed straight into
// MFMA f32 16x16x4 products against A = [-Dr -Ds -Dt | LIFT] (Appendix A,
// Eq. 10), then the fused low-storage RK stage update.  Members keep their
// own time, time step and inflow amplitude.  The persistent grid walks the
// concatenated element lists of all geometries; each XCD takes one
// contiguous range.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "batch.hpp"

namespace dg {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int N>
struct BShape {
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
  static constexpr int tabBytes = NF + 96 * Nfp + Np;
  static constexpr int total = KT * AS + (tabBytes + 15) / 16 * 4;  // floats: operator, tables
  static constexpr int slot = 5 * Np * kMembers;                     // one element's state
  // each wavefront stages its element's state in LDS when a block of
  // `waves` wavefronts still fits in the 160 KB of a CU
  static constexpr bool staged(int waves) { return (total + waves * slot) * 4 <= 160 * 1024; }
  static constexpr int lds_floats(int waves) { return total + (staged(waves) ? waves * slot : 0); }
  static_assert(slot % 4 == 0, "state block is whole 16-byte chunks");
};

template <class T>
__device__ __forceinline__ T pick4b(const T* x, int f) {
  return f == 0 ? x[0] : f == 1 ? x[1] : f == 2 ? x[2] : x[3];
}

// Global-address-space views: loads through them are global (not flat)
// loads, which the compiler does not count against LDS waits.
typedef __attribute__((address_space(1))) float gfloat;
__device__ __forceinline__ const gfloat* gview(const float* p) { return (const gfloat*)(p); }
__device__ __forceinline__ gfloat* gview(float* p) { return (gfloat*)(p); }

// Read-only tables through the constant address space: wave-uniform
// addresses become scalar loads.
typedef __attribute__((address_space(4))) const double cdouble;
typedef __attribute__((address_space(4))) const int cint;
typedef __attribute__((address_space(4))) const uint8_t cbyte;
typedef __attribute__((address_space(4))) const BatchGeom cgeom;

__device__ __forceinline__ cgeom& geom(const BatchLaunch& L, int gi) {
  return ((cgeom*)(L.geoms))[gi];
}

__device__ __forceinline__ float pulse(float amp, double alpha, double t) {
  const double T = 2.0 * M_PI / alpha;
  if (t >= 0.0 && t < T) return float(0.5 * amp * (1.0 - cos(alpha * t)));
  return 0.0f;
}

__device__ __forceinline__ int geom_of(const BatchLaunch& L, int64_t item) {
  int gi = 0;
  while (gi + 1 < L.ngeom && item >= geom(L, gi + 1).first) ++gi;
  return gi;
}

// per-member maximum over the 4 lane groups, then one atomic per member
__device__ __forceinline__ void flush_rate(const BatchLaunch& L, int gi, int lane, float& best,
                                           unsigned& bad) {
  best = fmaxf(best, __shfl_xor(best, 16));
  best = fmaxf(best, __shfl_xor(best, 32));
  bad |= __shfl_xor(bad, 16);
  bad |= __shfl_xor(bad, 32);
  const int e = lane & 15;
  if (lane < 16 && e < L.members) {
    BatchScalars* sc = geom(L, gi).sc;
    atomicMax(&sc->rate_bits[e], __float_as_uint(best));
    if (bad) atomicOr(&sc->bad[e], 1u);
  }
  best = 0.0f;
  bad = 0u;
}

__device__ __forceinline__ size_t qidx(int64_t k, int v, int node, int e, int Np) {
  return ((size_t(k) * 5 + v) * Np + node) * kMembers + e;
}

// LDS accesses of one wavefront are performed in order, but the compiler
// reasons per lane; the fences and the convergent wave barrier make a hand-off
// of LDS data between lanes explicit (no instruction on gfx950).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

typedef __attribute__((address_space(3))) void* lds_ptr_t;
typedef __attribute__((address_space(1))) void* gvoid_ptr_t;

template <int N, int WAVES>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(4))) void batch_stage_kernel(BatchLaunch L, float a_rk,
                                                                 float b_rk, double c_rk,
                                                                 int parity, int rate_out) {
  using S = BShape<N>;
  constexpr int Np = S::Np, Nfp = S::Nfp, MT = S::MT, AS = S::AS;
  constexpr bool STAGE = S::staged(WAVES);
  constexpr int QF = (Nfp + 3) / 4;  // face-node quads per face (the last padded)
  extern __shared__ float lds[];
  float* sA = lds;
  uint8_t* sFm = reinterpret_cast<uint8_t*>(lds + S::KT * AS);
  uint8_t* sNN = sFm + S::NF;
  uint8_t* sNF = sNN + 96 * Nfp;
  const Phys& P = L.phys;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int e = lane & 15;
  // this wavefront's copy of its element's state [5][Np][16] (staged form)
  float* sQ = lds + S::total + wave * S::slot;

  for (int i = tid; i < S::KT * AS; i += 64 * WAVES) sA[i] = L.Aop[i];
  for (int i = tid; i < S::NF; i += 64 * WAVES) sFm[i] = L.fmask[i];
  for (int i = tid; i < 96 * Nfp; i += 64 * WAVES) sNN[i] = L.nbr_node[i];
  for (int i = tid; i < Np; i += 64 * WAVES) sNF[i] = L.node_faces[i];
  __syncthreads();

  const int G = gridDim.x, nX = G < 8 ? G : 8;
  const int x = blockIdx.x % nX, jb = blockIdx.x / nX;
  const int Gx = G / nX + (x < G % nX ? 1 : 0);
  const int64_t c0 = L.total * x / nX, c1 = L.total * (x + 1) / nX;

  float rate_best = 0.0f;
  unsigned rate_bad = 0u;
  int gi = -1;
  int64_t first = 0, next_first = 0;
  float dt = 0.0f, pin = 0.0f;
  const gfloat* qi = nullptr;
  gfloat* qo = nullptr;
  gfloat* res = nullptr;
  const cdouble* vgeo = nullptr;
  const cdouble* sgeo = nullptr;
  const cint* nbrs = nullptr;
  const cbyte* finfo = nullptr;

  for (int64_t it = 0;; ++it) {
    const int64_t item = c0 + (int64_t(jb) + it * Gx) * WAVES + wave;
    if (item >= c1) break;
    if (gi < 0 || item >= next_first) {   // items ascend: the geometry only advances
      if (rate_out && gi >= 0) flush_rate(L, gi, lane, rate_best, rate_bad);
      gi = __builtin_amdgcn_readfirstlane(geom_of(L, item));
      cgeom& Gm = geom(L, gi);
      const double tm = Gm.sc->t[e] + c_rk * Gm.sc->dt[e];
      dt = float(Gm.sc->dt[e]);
      pin = pulse(Gm.amp[e], P.alpha, tm);
      qi = gview(Gm.q[parity]);
      qo = gview(Gm.q[1 - parity]);
      res = gview(Gm.res);
      vgeo = (const cdouble*)Gm.vgeo;
      sgeo = (const cdouble*)Gm.sgeo;
      nbrs = (const cint*)Gm.nbr;
      finfo = (const cbyte*)Gm.finfo;
      first = Gm.first;
      next_first = gi + 1 < L.ngeom ? geom(L, gi + 1).first : INT64_MAX;
    }
    const int64_t k = item - first;
    const gfloat* qk = qi + size_t(k) * 5 * Np * kMembers;
    // lane indices the compiler must treat as new each element: otherwise it
    // hoists every lane-dependent address and mask out of the element loop
    // and keeps them all live (spilling)
    int lane_t = lane;
    asm volatile("" : "+v"(lane_t));
    const int e = lane_t & 15, g = lane_t >> 4;
    const bool member = e < L.members;

    // own state: staged into LDS by asynchronous copies, or read from HBM
    if constexpr (STAGE) {
      wave_sync();                                  // every lane is done with the slot
      __builtin_amdgcn_s_waitcnt(0xc07f);           // and its LDS reads have returned
      constexpr int n4 = S::slot / 4;
#pragma unroll
      for (int j = 0; j < (n4 + 63) / 64; ++j) {
        const int i4 = j * 64 + lane;
        if (i4 < n4)
          __builtin_amdgcn_global_load_lds((gvoid_ptr_t)(qk + 4 * i4), (lds_ptr_t)(sQ + j * 256),
                                           16, 0, 0);
      }
    }
    auto own = [&](int v, int node) __attribute__((always_inline)) -> float {
      if constexpr (STAGE) return sQ[(v * Np + node) * kMembers + e];
      else return qk[(v * Np + node) * kMembers + e];
    };

    float gm[9], nx[4], ny[4], nz[4], fs[4];
    int nbr[4], finf[4];
#pragma unroll
    for (int i = 0; i < 9; ++i) gm[i] = float(vgeo[k * 9 + i]);
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      nx[f] = float(sgeo[k * 16 + f * 4 + 0]);
      ny[f] = float(sgeo[k * 16 + f * 4 + 1]);
      nz[f] = float(sgeo[k * 16 + f * 4 + 2]);
      fs[f] = float(sgeo[k * 16 + f * 4 + 3]);
      nbr[f] = nbrs[k * 4 + f];
      finf[f] = finfo[k * 4 + f];
    }

    // exterior traces of face f, lane (g, e) taking face nodes 4q + g of
    // member e; branch-free: boundary faces load the element's own trace and
    // discard it
    auto gather = [&](int f, float (&t)[QF][5]) __attribute__((always_inline)) {
      const int nb = pick4b(nbr, f), inf = pick4b(finf, f);
      const bool inner = nb >= 0;
#pragma unroll
      for (int q = 0; q < QF; ++q) {
        const int ii = min(4 * q + g, Nfp - 1);
        const int n2 = inner ? sNN[((f * 4 + (inf & 3)) * 6 + (inf >> 2)) * Nfp + ii]
                             : sFm[f * Nfp + ii];
        const gfloat* src = (inner ? qi + size_t(nb) * 5 * Np * kMembers : qk) + n2 * kMembers + e;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          const float val = src[v * Np * kMembers];
          t[q][v] = (inner && member) ? val : 0.0f;
        }
      }
    };
    if constexpr (STAGE) {
      __builtin_amdgcn_s_waitcnt(0);   // the staged state has landed
      wave_sync();
    }

    floatx4 acc[5][MT];
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[v][mt] = floatx4{0.f, 0.f, 0.f, 0.f};

    // volume
#pragma unroll 1
    for (int nq = 0; nq < S::NNQ; ++nq) {
      const int j = 4 * nq + g;
      float F[3][5];
      if (j < Np && member) {
        float q[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) q[v] = own(v, j);
        Prim w;
        primitive(P, q, w);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float d[3] = {gm[a * 3 + 0], gm[a * 3 + 1], gm[a * 3 + 2]};
          normal_flux(P, w, d, F[a]);
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
          for (int v = 0; v < 5; ++v)
            acc[v][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, F[a][v], acc[v][mt], 0, 0, 0);
        }
    }

    // faces one at a time (the exterior traces gathered per face: the kernel
    // runs four wavefronts per SIMD, which hide the gathers' latency better
    // than a register prefetch that would cost that occupancy): the face's
    // Lax-Friedrichs speed per member (max over its nodes and both sides,
    // reduced over the four lane groups), then the jump
    // Fscale/2 [n.(F- - F+) - lambda (q- - q+)] against the LIFT rows
#pragma unroll 1
    for (int f = 0; f < 4; ++f) {
      float trc[QF][5];
      gather(f, trc);
      const float n[3] = {pick4b(nx, f), pick4b(ny, f), pick4b(nz, f)};
      const int nb = pick4b(nbr, f);
      // the face's traces on both sides (recomputed in the two sub-passes
      // rather than kept alive across them)
      auto sides = [&](int q, float (&qm)[5], Prim& wm, float (&qp)[5], Prim& wp)
          __attribute__((always_inline)) {
        const int node = sFm[f * Nfp + min(4 * q + g, Nfp - 1)];
#pragma unroll
        for (int v = 0; v < 5; ++v) qm[v] = member ? own(v, node) : 0.0f;
        primitive(P, qm, wm);
        if (nb >= 0) {
#pragma unroll
          for (int v = 0; v < 5; ++v) qp[v] = trc[q][v];
        } else {
          ghost(P, -nb, qm, wm, n, pin, qp);
        }
        primitive(P, qp, wp);
      };
      float lam = 0.0f;
#pragma unroll
      for (int q = 0; q < QF; ++q) {
        float qm[5], qp[5];
        Prim wm, wp;
        sides(q, qm, wm, qp, wp);
        const float sp = fmaxf(normal_speed(P, wm, n), normal_speed(P, wp, n));
        if (4 * q + g < Nfp) lam = fmaxf(lam, sp);
      }
      lam = fmaxf(lam, __shfl_xor(lam, 16));
      lam = fmaxf(lam, __shfl_xor(lam, 32));
      const float hs = member ? 0.5f * pick4b(fs, f) : 0.0f;
#pragma unroll
      for (int q = 0; q < QF; ++q) {
        const int ii = 4 * q + g;
        float qm[5], qp[5], fm[5], fp[5], dF[5];
        Prim wm, wp;
        sides(q, qm, wm, qp, wp);
        normal_flux(P, wm, n, fm);
        normal_flux(P, wp, n, fp);
        const float h = ii < Nfp ? hs : 0.0f;
#pragma unroll
        for (int v = 0; v < 5; ++v) dF[v] = h * ((fm[v] - fp[v]) - lam * (qm[v] - qp[v]));
        const int row = S::KV + f * Nfp + min(ii, Nfp - 1);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const float av = sA[row * AS + mt * 16 + e];
#pragma unroll
          for (int v = 0; v < 5; ++v)
            acc[v][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, dF[v], acc[v][mt], 0, 0, 0);
        }
      }
    }

    // epilogue: lane holds nodes mt*16 + 4g + r of member e, all variables;
    // the residuals are loaded together first
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int node = mt * 16 + 4 * g + r;
        if (node >= Np || !member) continue;
        float qn[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          const size_t gx = qidx(k, v, node, e, Np);
          const float rr = dt * acc[v][mt][r] + (a_rk != 0.0f ? a_rk * res[gx] : 0.0f);
          res[gx] = rr;
          qn[v] = own(v, node) + b_rk * rr;
          qo[gx] = qn[v];
        }
        if (rate_out) {
          const int faces = sNF[node];
          if (faces) {
            float fmax = 0.0f;
#pragma unroll
            for (int ff = 0; ff < 4; ++ff)
              if (faces & (1 << ff)) fmax = fmaxf(fmax, fs[ff]);
            Prim w;
            primitive(P, qn, w);
            float u2 = 0.0f;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              const float u = P.u0[d] + w.du[d];
              u2 += u * u;
            }
            const float rate = P.half_N1sq * fmax * (sqrtf(u2) + sqrtf(P.gamma * w.p / w.rho));
            if (!(w.rho > 0.0f) || !(w.p > 0.0f) || !(rate == rate)) rate_bad = 1u;
            else rate_best = fmaxf(rate_best, rate);
          }
        }
      }
  }
  if (rate_out && gi >= 0) flush_rate(L, gi, lane, rate_best, rate_bad);
}

// CFL rate of the start state: max over face nodes of (N+1)^2/2 Fscale (|u|+c)
template <int N>
__global__ __launch_bounds__(256) void batch_rate_kernel(BatchLaunch L, int parity) {
  using S = BShape<N>;
  constexpr int Np = S::Np, Nfp = S::Nfp;
  const int tid = threadIdx.x, lane = tid & 63, e = lane & 15, g = lane >> 4;
  const bool member = e < L.members;
  const Phys& P = L.phys;
  float best = 0.0f;
  unsigned bad = 0u;
  int cur = -1;
  for (int64_t item = (int64_t(blockIdx.x) * 256 + tid) / 64; item < L.total;
       item += int64_t(gridDim.x) * 4) {
    const int gi = geom_of(L, item);
    if (gi != cur) {
      if (cur >= 0) flush_rate(L, cur, lane, best, bad);
      cur = gi;
    }
    cgeom& Gm = geom(L, gi);
    const int64_t k = item - Gm.first;
    const float* qi = Gm.q[parity];
    for (int fq = 0; fq < S::NFQ; ++fq) {
      const int i = 4 * fq + g, f = i / Nfp;
      const int node = L.fmask[i];
      float q[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) q[v] = member ? qi[qidx(k, v, node, e, Np)] : 0.0f;
      Prim w;
      primitive(P, q, w);
      float u2 = 0.0f;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const float u = P.u0[d] + w.du[d];
        u2 += u * u;
      }
      const float rate = P.half_N1sq * float(Gm.sgeo[k * 16 + f * 4 + 3]) *
                         (sqrtf(u2) + sqrtf(P.gamma * w.p / w.rho));
      if (!(w.rho > 0.0f) || !(w.p > 0.0f) || !(rate == rate)) bad = 1u;
      else best = fmaxf(best, rate);
    }
  }
  if (cur >= 0) flush_rate(L, cur, lane, best, bad);
}

__global__ void batch_finalize_kernel(BatchLaunch L) {
  const int gi = blockIdx.x, e = threadIdx.x;
  if (gi >= L.ngeom || e >= L.members) return;
  BatchScalars* sc = geom(L, gi).sc;
  const float rate = __uint_as_float(sc->rate_bits[e]);
  sc->dt[e] = rate > 0.0f ? sc->cfl / double(rate) : 0.0;
  if (sc->bad[e] && sc->first_bad[e] < 0) sc->first_bad[e] = sc->step;
  sc->rate_bits[e] = 0u;
  sc->bad[e] = 0u;
}

__global__ void batch_advance_kernel(BatchLaunch L) {
  const int gi = blockIdx.x, e = threadIdx.x;
  if (gi >= L.ngeom || e >= L.members) return;
  BatchScalars* sc = geom(L, gi).sc;
  sc->t[e] += sc->dt[e];
  if (e == 0) sc->step += 1;
}

template <int N, int W>
hipError_t prep(int* bpc) {
  const int lds = int(BShape<N>::lds_floats(W) * sizeof(float));
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&batch_stage_kernel<N, W>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  int nb = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &nb, reinterpret_cast<const void*>(&batch_stage_kernel<N, W>), 64 * W, lds);
  if (e == hipSuccess) *bpc = std::max(nb, 1);
  return e;
}

template <int N>
hipError_t prep_n(int waves, int* bpc) {
  switch (waves) {
    case 1: return prep<N, 1>(bpc);
    case 2: return prep<N, 2>(bpc);
    case 4: return prep<N, 4>(bpc);
    case 8: return prep<N, 8>(bpc);
    default: return hipErrorInvalidValue;
  }
}

template <int N, int W>
void launch_w(const BatchLaunch& L, float a, float b, double c, int parity, int rate_out,
              hipStream_t s) {
  const int64_t want = (L.total + W - 1) / W;
  const int blocks = int(std::max<int64_t>(1, std::min<int64_t>(want, int64_t(L.num_cu) * L.blocks_per_cu)));
  const size_t lds = size_t(BShape<N>::lds_floats(W)) * sizeof(float);
  batch_stage_kernel<N, W><<<blocks, 64 * W, lds, s>>>(L, a, b, c, parity, rate_out);
}

template <int N>
void launch_n(const BatchLaunch& L, float a, float b, double c, int parity, int rate_out,
              hipStream_t s) {
  switch (L.waves_per_block) {
    case 1: launch_w<N, 1>(L, a, b, c, parity, rate_out, s); break;
    case 2: launch_w<N, 2>(L, a, b, c, parity, rate_out, s); break;
    case 8: launch_w<N, 8>(L, a, b, c, parity, rate_out, s); break;
    default: launch_w<N, 4>(L, a, b, c, parity, rate_out, s); break;
  }
}

}  // namespace

hipError_t prepare_batch_kernels(int N, int waves_per_block, int* blocks_per_cu) {
  switch (N) {
    case 1: return prep_n<1>(waves_per_block, blocks_per_cu);
    case 2: return prep_n<2>(waves_per_block, blocks_per_cu);
    case 3: return prep_n<3>(waves_per_block, blocks_per_cu);
    case 4: return prep_n<4>(waves_per_block, blocks_per_cu);
    case 5: return prep_n<5>(waves_per_block, blocks_per_cu);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_batch_stage(const BatchLaunch& L, float a, float b, double c, int parity,
                              int rate_out, hipStream_t s) {
  switch (L.N) {
    case 1: launch_n<1>(L, a, b, c, parity, rate_out, s); break;
    case 2: launch_n<2>(L, a, b, c, parity, rate_out, s); break;
    case 3: launch_n<3>(L, a, b, c, parity, rate_out, s); break;
    case 4: launch_n<4>(L, a, b, c, parity, rate_out, s); break;
    case 5: launch_n<5>(L, a, b, c, parity, rate_out, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch_rate(const BatchLaunch& L, int parity, hipStream_t s) {
  const int blocks = int(std::max<int64_t>(1, std::min<int64_t>((L.total + 3) / 4, 4096)));
  switch (L.N) {
    case 1: batch_rate_kernel<1><<<blocks, 256, 0, s>>>(L, parity); break;
    case 2: batch_rate_kernel<2><<<blocks, 256, 0, s>>>(L, parity); break;
    case 3: batch_rate_kernel<3><<<blocks, 256, 0, s>>>(L, parity); break;
    case 4: batch_rate_kernel<4><<<blocks, 256, 0, s>>>(L, parity); break;
    case 5: batch_rate_kernel<5><<<blocks, 256, 0, s>>>(L, parity); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch_finalize(const BatchLaunch& L, hipStream_t s) {
  batch_finalize_kernel<<<L.ngeom, kMembers, 0, s>>>(L);
  return hipGetLastError();
}

hipError_t launch_batch_advance(const BatchLaunch& L, hipStream_t s) {
  batch_advance_kernel<<<L.ngeom, kMembers, 0, s>>>(L);
  return hipGetLastError();
}

}  // namespace dg
