// HIP kernels of the nodal DG Euler hot path (gfx950 / CDNA4).
//
// Fused stage kernel.  A block of four wavefronts owns a tile of 16
// consecutive elements at a time (persistent grid; each of the 8 XCDs sweeps
// a contiguous range of tiles so that neighbour traces mostly hit its L2):
//   A. the tile's state q' [16][5][Np] (asynchronous global->LDS copies) and
//      every exterior face trace it needs (into the registers of the lane
//      that uses it; LDS copies in the split-BF16 form) are requested at once,
//      so the neighbour gathers never stall a wavefront one face at a time;
//   B. the local Lax-Friedrichs speed of each element face,
//      max over its nodes and both sides of |u.n| + c, is reduced in LDS;
//   C. the contraction is split over the four wavefronts along its length:
//      each lane forms the flux of one (node, element) pair -- contravariant
//      fluxes r_x F + r_y G + r_z H etc. for the volume term, the
//      Lax-Friedrichs jump [n.(F- - F+) - lambda (q- - q+)] Fscale / 2 for the
//      surface term (Appendix A, Eq. 10) -- and feeds it straight into the B
//      operand of MFMA f32 16x16x4 products against A = [-Dr -Ds -Dt | LIFT],
//      one accumulator set per conserved variable;
//   D. the four partial sums are added in a fixed order (bitwise
//      reproducible) and the epilogue writes rhs or the fused low-storage RK
//      stage update with coalesced accesses.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "kernels.hpp"

namespace dg {
namespace {

constexpr int kTileE = 16;  // elements per tile (MFMA n = 16)
constexpr int kWaves = 4;   // wavefronts per block
constexpr int kThreads = 64 * kWaves;

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void* lds_ptr_t;

enum : int { PREC_FP32 = 0, PREC_BF16 = 1 };

template <int N, int PREC = PREC_FP32>
struct Shape {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
  static constexpr int NF = 4 * Nfp;              // face nodes per element
  static constexpr int NFQ = NF / 4;              // face-node quads
  static constexpr int NNQ = (Np + 3) / 4;        // node quads
  static constexpr int NQP = 4 * NNQ;             // nodes padded to quads
  static constexpr int KV = 3 * NQP;              // volume contraction rows
  static constexpr int KT = KV + NF;              // all contraction rows
  static constexpr int MP = (Np + 15) / 16 * 16;  // output rows padded to 16
  static constexpr int MT = MP / 16;
  static constexpr int AS = (MP % 32 == 16) ? MP : MP + 16;  // row stride of A
  static constexpr int ST = 5 * Np;               // floats per element state
  // split-BF16 volume: k-blocks of 32 = 4 lane groups x (2 nodes x 3
  // directions + 2 zero pads); the operator halves hi, lo are [MP][KVB]
  static constexpr int NKB = (Np + 7) / 8;
  static constexpr int KVB = 32 * NKB;
  // rows of the FP32 operator kept in LDS: all, or the LIFT rows only
  static constexpr int AROW0 = (PREC == PREC_BF16) ? KV : 0;
  static constexpr bool A_LDS = (KT - AROW0) * AS * 4 <= 40 * 1024;
  static constexpr int tabFloats = (NF + 96 * Nfp + 15) / 16 * 4;
  static constexpr int MPS = MP + 4;  // padded row of a partial sum (conflict-free 16-byte writes)
  static constexpr int scratch = (NF * 5 * kTileE > kWaves * kTileE * MPS) ? NF * 5 * kTileE
                                                                            : kWaves * kTileE * MPS;
  // LDS layout (floats)
  static constexpr int oA = 0;
  static constexpr int oTab = oA + (A_LDS ? (KT - AROW0) * AS : 0);
  static constexpr int oQ = oTab + tabFloats;        // [16][5][Np] state tile
  static constexpr int oR = oQ + kTileE * ST;        // [16][5][Np] residual tile
  static constexpr int oP = oR + kTileE * ST;        // exterior traces / reduction
  // FP32 geometry of the tile, component-major [25][16]: the metric terms
  // d(r,s,t)/d(x,y,z) (components 0..8), then nx, ny, nz, Fscale of each face
  static constexpr int oG = oP + scratch;
  static constexpr int oL = oG + kTileE * 25;        // [16][4] face speeds
  static_assert(oG % 4 == 0, "16-byte chunks of the geometry copy");
  // split-BF16: n.(F- - F+) gets its own region and q- - q+ is recomputed
  // (frees registers for the BF16 operands)
  static constexpr bool DQ_LDS = PREC == PREC_BF16;
  static constexpr int oD = oL + kTileE * 4;         // [NF quads][5][64]
  static constexpr int total = oD + (DQ_LDS ? NF * 5 * kTileE : 0);
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

// x[f] for a runtime face index f in 0..3 held in registers (selects, no
// dynamic register indexing)
template <class T>
__device__ __forceinline__ T pick4(const T* x, int f) {
  return f == 0 ? x[0] : f == 1 ? x[1] : f == 2 ? x[2] : x[3];
}

__device__ __forceinline__ floatx4 mfma(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ floatx4 mfma_bf16(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// x = hi + lo + O(2^-16 |x|): hi = bf16(x), lo = bf16(x - hi), round to nearest even
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

// EXTRA: bit 0 an absorbing layer (rhs -= sigma q'), bit 1 a curved set
// (its elements' outputs and rate are left to the curved pass); plain meshes
// run the kernel with neither.
enum : int { EXTRA_DAMP = 1, EXTRA_CURVED = 2 };

template <int N, int MODE, bool MOVING, int PREC, int EXTRA>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void stage_kernel(DeviceMesh m, const float* __restrict__ q_in,
                                                         float* __restrict__ q_out,
                                                         float* __restrict__ res,
                                                         float* __restrict__ out, float a_rk,
                                                         float b_rk, double c_rk, double t_host,
                                                         double dt_host, RunScalars* run,
                                                         int rate_out) {
  using S = Shape<N, PREC>;
  constexpr int Np = S::Np, Nfp = S::Nfp, ST = S::ST, MT = S::MT, AS = S::AS, MP = S::MP;
  constexpr bool DAMP = (EXTRA & EXTRA_DAMP) != 0, CURVED = (EXTRA & EXTRA_CURVED) != 0;
  extern __shared__ float lds[];
  // row k of the FP32 operator is sA[k * AS + col] (LDS holds rows >= AROW0)
  const float* sA = S::A_LDS ? lds + S::oA - S::AROW0 * AS : m.Aop;
  uint8_t* sFm = reinterpret_cast<uint8_t*>(lds + S::oTab);
  uint8_t* sNN = sFm + S::NF;
  float* sQ = lds + S::oQ;
  float* sR = lds + S::oR;
  float* sP = lds + S::oP;
  const float* sGe = lds + S::oG;       // [25][16] geometry: component c of element e at c*16 + e
  unsigned* sL = reinterpret_cast<unsigned*>(lds + S::oL);
  const Phys& P = m.phys;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int e = lane & 15, g = lane >> 4;

  if (S::A_LDS)
    for (int i = tid; i < (S::KT - S::AROW0) * AS; i += kThreads)
      lds[S::oA + i] = m.Aop[S::AROW0 * AS + i];
  for (int i = tid; i < S::NF; i += kThreads) sFm[i] = m.fmask[i];
  for (int i = tid; i < 96 * Nfp; i += kThreads) sNN[i] = m.nbr_node[i];

  const double tst = stage_time(c_rk, t_host, dt_host, run);
  const float pin = inflow_pressure(P, tst);
  const float dt = float(run ? run->dt : dt_host);

  const int64_t ntiles = (m.K + kTileE - 1) / kTileE;
  const int G = gridDim.x, nX = G < 8 ? G : 8;
  const int x = blockIdx.x % nX, jb = blockIdx.x / nX;
  const int Gx = G / nX + (x < G % nX ? 1 : 0);
  const int64_t c0 = ntiles * x / nX, c1 = ntiles * (x + 1) / nX;

  // connectivity of a lane's element, one tile ahead: 4 neighbours + packed
  // (neighbour face | orientation << 2) bytes, and (CURVED) whether the
  // element is curved
  auto load_conn = [&](int64_t t, int4& nb4, unsigned& fi4, int& cf) {
    const int64_t kk = t * kTileE + e;
    cf = 0;
    if (t < c1 && kk < m.K) {
      nb4 = reinterpret_cast<const int4*>(m.nbr)[kk];
      fi4 = reinterpret_cast<const unsigned*>(m.finfo)[kk];
      if (CURVED) cf = m.curved_flag[kk];
    } else {
      nb4 = make_int4(-BC_PASSTHRU, -BC_PASSTHRU, -BC_PASSTHRU, -BC_PASSTHRU);
      fi4 = 0u;
    }
  };
  int4 nbN;
  unsigned fiN;
  int cfN;
  load_conn(c0 + jb, nbN, fiN, cfN);
  constexpr int kOut = (kTileE * MP + kThreads - 1) / kThreads;
  constexpr int kFQ = (S::NFQ + kWaves - 1) / kWaves;

  // exterior-trace offsets (neighbour element * ST + node) of this lane's
  // face quads, or -1 on boundary faces; computed one tile ahead so that the
  // gathers are issued without an LDS table read in front of them
  int goff[kFQ];
  auto gather_offsets = [&](int64_t t) {
    const bool ok = t < c1 && t * kTileE + e < m.K;
    const int nbv[4] = {nbN.x, nbN.y, nbN.z, nbN.w};
#pragma unroll
    for (int kq = 0; kq < kFQ; ++kq) {
      const int fq = w + kWaves * kq;
      const int i = 4 * fq + g, f = i / Nfp, ii = i - f * Nfp;
      const int nb = pick4(nbv, f);
      int off = -1;
      if (ok && fq < S::NFQ && nb >= 0) {
        const int inf = (fiN >> (8 * f)) & 0xff;
        off = nb * ST + sNN[((f * 4 + (inf & 3)) * 6 + (inf >> 2)) * Nfp + ii];
      } else if (ok && fq < S::NFQ && m.lghost && ((-nb) & 7) == BC_LEARNED) {
        off = -2 - (((-nb) >> 3) * ST + ii);  // learned ghost trace, same layout
      }
      goff[kq] = off;
    }
  };
  __syncthreads();  // tables in LDS
  gather_offsets(c0 + jb);

  float rate_best = 0.0f;   // time-step reduction over this block's tiles
  unsigned rate_bad = 0u;
  // FP32: the exterior traces go straight into the registers of the lane
  // that uses them in the surface pass (the split-BF16 form re-reads them
  // from LDS in the contraction pass, so it stages them there)
  constexpr bool TR_REG = PREC == PREC_FP32;
  float trv[TR_REG ? kFQ : 1][5];
  for (int64_t tile = c0 + jb; tile < c1; tile += Gx) {
    // at N >= 5, thread indices the compiler must treat as new each tile:
    // otherwise it hoists every lane-dependent address out of the tile loop
    // and keeps them all live (spilling); at lower orders the hoisting fits
    // in registers and is the faster schedule
    int tid_t = tid;
    if constexpr (N >= 5) asm volatile("" : "+v"(tid_t));
    const int lane = tid_t & 63, e = lane & 15, g = lane >> 4;
    const int64_t k0 = tile * kTileE;
    const int ne = int(min<int64_t>(kTileE, m.K - k0));
    const bool valid = e < ne;
    const int nbr[4] = {nbN.x, nbN.y, nbN.z, nbN.w};
    // (CURVED) the tile's curved elements, bit e: their outputs and rate are
    // the curved pass's
    const unsigned cmask = CURVED ? unsigned(__ballot(cfN != 0)) & 0xffffu : 0u;
    __syncthreads();  // previous tile fully consumed (and prologue tables ready)

    // A. asynchronous loads: exterior traces (offsets precomputed), then the
    // state and residual tiles and the FP64 geometry
    if (tid_t < kTileE * 4) sL[tid_t] = 0u;
#pragma unroll
    for (int kq = 0; kq < kFQ; ++kq) {
      const int fq = w + kWaves * kq;
      if (TR_REG) {
        // (no load on boundary faces: goff = -1 points the address at q_in)
        const float* src = goff[kq] >= 0 ? q_in + goff[kq]
                           : (goff[kq] < -1 ? m.lghost + (-2 - goff[kq]) : q_in);
#pragma unroll
        for (int v = 0; v < 5; ++v) trv[TR_REG ? kq : 0][v] = goff[kq] != -1 ? src[v * Np] : 0.0f;
      } else if (goff[kq] != -1) {
        const float* src = goff[kq] >= 0 ? q_in + goff[kq] : m.lghost + (-2 - goff[kq]);
#pragma unroll
        for (int v = 0; v < 5; ++v)
          __builtin_amdgcn_global_load_lds((void*)(src + v * Np), (lds_ptr_t)(sP + (fq * 5 + v) * 64),
                                           4, 0, 0);
      }
    }
    // state and residual tiles, FP64 geometry
    const float* qg = q_in + k0 * ST;
    const bool want_res = MODE == MODE_STAGE && a_rk != 0.0f;
    if (ne == kTileE) {
      constexpr int n4 = kTileE * ST / 4;
      for (int j = w; j * 64 < n4; j += kWaves) {
        const int i4 = j * 64 + lane;
        if (i4 < n4) {
          __builtin_amdgcn_global_load_lds((void*)(qg + 4 * i4), (lds_ptr_t)(sQ + j * 256), 16, 0, 0);
          if (want_res)
            __builtin_amdgcn_global_load_lds((void*)(res + k0 * ST + 4 * i4),
                                             (lds_ptr_t)(sR + j * 256), 16, 0, 0);
        }
      }
      // FP32 geometry of the tile, already in its LDS layout: 1600
      // contiguous bytes, 16-byte chunks
      if (w == kWaves - 1) {
        const char* gsrc = reinterpret_cast<const char*>(m.geo32 + tile * kTileE * 25);
        char* gdst = reinterpret_cast<char*>(lds + S::oG);
        __builtin_amdgcn_global_load_lds((void*)(gsrc + 16 * lane), (lds_ptr_t)(gdst), 16, 0, 0);
        if (lane < 36)
          __builtin_amdgcn_global_load_lds((void*)(gsrc + 1024 + 16 * lane), (lds_ptr_t)(gdst + 1024),
                                           16, 0, 0);
      }
    } else {
      for (int i = tid_t; i < kTileE * ST; i += kThreads) {
        sQ[i] = (i < ne * ST) ? qg[i] : 0.0f;
        if (want_res) sR[i] = (i < ne * ST) ? res[k0 * ST + i] : 0.0f;
      }
      // (the geometry array is zero past the last element)
      for (int i = tid_t; i < kTileE * 25; i += kThreads) lds[S::oG + i] = m.geo32[tile * kTileE * 25 + i];
    }
    load_conn(tile + Gx, nbN, fiN, cfN);  // next tile's connectivity, in flight meanwhile
    __builtin_amdgcn_s_waitcnt(0);
    gather_offsets(tile + Gx);
    __syncthreads();

    // B. surface: traces, face speeds and the normal-flux difference
    //    n.(F- - F+) (stored over the staged exterior trace); q- - q+ stays
    //    in registers for the contraction pass (same lanes, same quads)
    float dq[S::DQ_LDS ? 1 : kFQ][5];
    float* sD = lds + S::oD;
#pragma unroll
    for (int kq = 0; kq < kFQ; ++kq) {
      const int fq = w + kWaves * kq;
      if (fq >= S::NFQ) break;
      const int i = 4 * fq + g, f = i / Nfp;
      const float n[3] = {sGe[(9 + f * 4) * kTileE + e], sGe[(10 + f * 4) * kTileE + e],
                          sGe[(11 + f * 4) * kTileE + e]};
      const int node = sFm[i];
      float qm[5], qp[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) qm[v] = sQ[e * ST + v * Np + node];
      Prim wm;
      primitive<MOVING>(P, qm, wm);
      const int nb = valid ? pick4(nbr, f) : -BC_PASSTHRU;
      float* slot = sP + fq * 5 * 64 + lane;
      if (nb >= 0 || (m.lghost && ((-nb) & 7) == BC_LEARNED)) {
#pragma unroll
        for (int v = 0; v < 5; ++v) qp[v] = TR_REG ? trv[TR_REG ? kq : 0][v] : slot[v * 64];
      } else {
        ghost(P, -nb, qm, wm, n, pin, qp);
      }
      Prim wp;
      primitive<MOVING>(P, qp, wp);
      const float lam = fmaxf(normal_speed<MOVING>(P, wm, n), normal_speed<MOVING>(P, wp, n));
      if (valid) atomicMax(&sL[e * 4 + f], __float_as_uint(lam));
      float fm[5], fp[5];
      normal_flux<MOVING>(P, wm, n, fm);
      normal_flux<MOVING>(P, wp, n, fp);
      if (S::DQ_LDS) {
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          sD[fq * 5 * 64 + lane + v * 64] = fm[v] - fp[v];
          if (nb < 0) slot[v * 64] = qp[v];  // ghost state, for the recomputation
        }
      } else {
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          slot[v * 64] = fm[v] - fp[v];
          dq[kq][v] = qm[v] - qp[v];
        }
      }
    }
    __syncthreads();

    // C. contraction, split over the wavefronts
    floatx4 acc[5][MT];
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[v][mt] = floatx4{0.f, 0.f, 0.f, 0.f};

    float gm[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) gm[i] = sGe[i * kTileE + e];
    if (PREC == PREC_BF16) {
      // volume on BF16 MFMA: D (hi, lo) x F' (hi, lo), lo*lo dropped
      const bf16x8* Ab = reinterpret_cast<const bf16x8*>(m.Abf);
      for (int kb = w; kb < S::NKB; kb += kWaves) {
        float F[2][3][5];
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
          const int j = 8 * kb + 2 * g + jj;
          if (j < Np && valid) {
            float q[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) q[v] = sQ[e * ST + v * Np + j];
            Prim wv;
            primitive<MOVING>(P, q, wv);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const float d[3] = {gm[a * 3 + 0], gm[a * 3 + 1], gm[a * 3 + 2]};
              normal_flux<MOVING>(P, wv, d, F[jj][a]);
            }
          } else {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
              for (int v = 0; v < 5; ++v) F[jj][a][v] = 0.0f;
          }
        }
        bf16x8 Ahi[MT], Alo[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int row = mt * 16 + e;
          Ahi[mt] = Ab[(row * S::KVB + kb * 32 + 8 * g) / 8];
          Alo[mt] = Ab[((MP + row) * S::KVB + kb * 32 + 8 * g) / 8];
        }
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          bf16x8 Bhi, Blo;
#pragma unroll
          for (int jj = 0; jj < 2; ++jj)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              __bf16 h, l;
              split_bf16(F[jj][a][v], h, l);
              Bhi[3 * jj + a] = h;
              Blo[3 * jj + a] = l;
            }
          Bhi[6] = Bhi[7] = Blo[6] = Blo[7] = (__bf16)0.0f;
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            acc[v][mt] = mfma_bf16(Ahi[mt], Bhi, acc[v][mt]);
            acc[v][mt] = mfma_bf16(Ahi[mt], Blo, acc[v][mt]);
            acc[v][mt] = mfma_bf16(Alo[mt], Bhi, acc[v][mt]);
          }
        }
      }
    } else {
      for (int nq = (w + 1) % kWaves; nq < S::NNQ; nq += kWaves) {
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
    }

    // surface term: dF = Fscale/2 [n.(F- - F+) - lambda (q- - q+)]
#pragma unroll
    for (int kq = 0; kq < kFQ; ++kq) {
      const int fq = w + kWaves * kq;
      if (fq >= S::NFQ) break;
      const int i = 4 * fq + g, f = i / Nfp;
      const float lam = __uint_as_float(sL[e * 4 + f]);
      const float hs = valid ? 0.5f * sGe[(12 + f * 4) * kTileE + e] : 0.0f;
      const float* slot = sP + fq * 5 * 64 + lane;
      float dF[5];
      if (S::DQ_LDS) {
        const int node = sFm[i];
#pragma unroll
        for (int v = 0; v < 5; ++v)
          dF[v] = hs * (sD[fq * 5 * 64 + lane + v * 64] -
                        lam * (sQ[e * ST + v * Np + node] - slot[v * 64]));
      } else {
#pragma unroll
        for (int v = 0; v < 5; ++v) dF[v] = hs * (slot[v * 64] - lam * dq[kq][v]);
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const float av = sA[(S::KV + i) * AS + mt * 16 + e];
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[v][mt] = mfma(av, dF[v], acc[v][mt]);
      }
    }

    // D. fixed-order reduction of the four partial sums, then the epilogue
    // (with an absorbing layer, the rates of this thread's outputs, loaded
    // once for all five variables)
    float sig[DAMP ? kOut : 1];
    if (DAMP) {
#pragma unroll
      for (int i = 0; i < kOut; ++i) {
        const int o = min(tid_t + i * kThreads, kTileE * MP - 1);
        const int eo = o / MP, node = o - eo * MP;
        sig[i] = (eo < ne && node < Np) ? m.sigma[(k0 + eo) * Np + node] : 0.0f;
      }
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      __syncthreads();  // sP free (traces consumed / previous round read)
      // partial sums transposed to [wave][element][node]: lane (g, e) holds
      // nodes mt*16 + 4g .. +3 of element e
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
        *reinterpret_cast<floatx4*>(sP + (w * kTileE + e) * S::MPS + mt * 16 + 4 * g) = acc[v][mt];
      __syncthreads();
      float sum[kOut], qv[kOut], rv[kOut];
      int64_t gidx[kOut];
      bool okv[kOut];
#pragma unroll
      for (int i = 0; i < kOut; ++i) {
        const int o = min(tid_t + i * kThreads, kTileE * MP - 1);
        const int eo = o / MP, node = o - eo * MP;
        okv[i] = (tid_t + i * kThreads < kTileE * MP) && node < Np && eo < ne &&
                 !(CURVED && ((cmask >> eo) & 1u));
        const int nd = node < Np ? node : Np - 1;
        float acc_s = 0.0f;
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) acc_s += sP[(ww * kTileE + eo) * S::MPS + node];
        sum[i] = acc_s;
        qv[i] = sQ[eo * ST + v * Np + nd];
        // absorbing layer: relaxation of q' towards zero at the node's rate
        if (DAMP) sum[i] -= sig[DAMP ? i : 0] * qv[i];
        rv[i] = (MODE == MODE_STAGE && a_rk != 0.0f) ? sR[eo * ST + v * Np + nd] : 0.0f;
        gidx[i] = (k0 + eo) * ST + v * Np + nd;
      }
#pragma unroll
      for (int i = 0; i < kOut; ++i) {
        if (!okv[i]) continue;
        if (MODE == MODE_RHS) {
          out[gidx[i]] = sum[i];
        } else {
          const float rr = dt * sum[i] + a_rk * rv[i];
          const float qn = qv[i] + b_rk * rr;
          res[gidx[i]] = rr;
          q_out[gidx[i]] = qn;
          if (rate_out) {  // same thread, same element/variable/node: in place
            const int o = tid_t + i * kThreads;
            const int eo = o / MP, node = o - eo * MP;
            sQ[eo * ST + v * Np + node] = qn;
          }
        }
      }
    }

    // time-step rule for the next step, from the new state (last stage only):
    // max over face nodes of (N+1)^2/2 Fscale (|u| + c); non-physical states flagged
    if (MODE == MODE_STAGE && rate_out) {
      __syncthreads();
      for (int it = tid_t; it < kTileE * S::NF; it += kThreads) {
        const int eo = it / S::NF, i = it - eo * S::NF, f = i / Nfp;
        if (eo >= ne || (CURVED && ((cmask >> eo) & 1u))) continue;
        const int node = sFm[i];
        float qq[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) qq[v] = sQ[eo * ST + v * Np + node];
        Prim wv;
        primitive<MOVING>(P, qq, wv);
        float sp2 = 0.0f;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const float u = P.u0[d] + wv.du[d];
          sp2 += u * u;
        }
        const float rate = P.half_N1sq * sGe[(12 + f * 4) * kTileE + eo] *
                           (sqrtf(sp2) + sqrtf(P.gamma * wv.p / wv.rho));
        if (!(wv.rho > 0.0f) || !(wv.p > 0.0f) || !(rate == rate)) rate_bad = 1u;
        else rate_best = fmaxf(rate_best, rate);
      }
    }
  }

  if (MODE == MODE_STAGE && rate_out) {
    // one atomic per block: wavefront max, then across the block's wavefronts
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      rate_best = fmaxf(rate_best, __shfl_xor(rate_best, off));
      rate_bad |= __shfl_xor(rate_bad, off);
    }
    __syncthreads();
    if (lane == 0) {
      sL[2 * w] = __float_as_uint(rate_best);
      sL[2 * w + 1] = rate_bad;
    }
    __syncthreads();
    if (tid == 0) {
      float b = 0.0f;
      unsigned bd = 0u;
      for (int ww = 0; ww < kWaves; ++ww) {
        b = fmaxf(b, __uint_as_float(sL[2 * ww]));
        bd |= sL[2 * ww + 1];
      }
      atomicMax(&run->rate_bits, __float_as_uint(b));
      if (bd) atomicOr(&run->bad, 1u);
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
  // wavefront max, block max, then one atomic per block (order-independent;
  // one per wave would serialize tens of thousands of atomics on one word)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    best = fmaxf(best, __shfl_xor(best, off));
    bad |= __shfl_xor(bad, off);
  }
  __shared__ float wbest[4];
  __shared__ unsigned wbad[4];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    wbest[w] = best;
    wbad[w] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const float b = fmaxf(fmaxf(wbest[0], wbest[1]), fmaxf(wbest[2], wbest[3]));
    atomicMax(&run->rate_bits, __float_as_uint(b));
    if (wbad[0] | wbad[1] | wbad[2] | wbad[3]) atomicOr(&run->bad, 1u);
  }
}

// one block of kRateParts threads (rates are non-negative, so the largest
// float is the largest bit pattern)
__global__ __launch_bounds__(kRateParts) void finalize_kernel(RunScalars* run) {
  __shared__ unsigned wmax[kRateParts / 64];
  unsigned b = run->rate_part[threadIdx.x];
  run->rate_part[threadIdx.x] = 0u;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) b = max(b, unsigned(__shfl_xor(int(b), off)));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = b;
  __syncthreads();
  if (threadIdx.x != 0) return;
  unsigned bits = run->rate_bits;
  for (int w = 0; w < kRateParts / 64; ++w) bits = max(bits, wmax[w]);
  const float rate = __uint_as_float(bits);
  run->dt = run->fixed_dt > 0.0 ? run->fixed_dt : (rate > 0.0f) ? run->cfl / double(rate) : 0.0;
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

template <int N, int MODE, bool MOVING, int PREC>
hipError_t set_lds_limit() {
  const int lds = int(Shape<N, PREC>::total * sizeof(float));
  const void* fns[4] = {reinterpret_cast<const void*>(&stage_kernel<N, MODE, MOVING, PREC, 0>),
                        reinterpret_cast<const void*>(&stage_kernel<N, MODE, MOVING, PREC, 1>),
                        reinterpret_cast<const void*>(&stage_kernel<N, MODE, MOVING, PREC, 2>),
                        reinterpret_cast<const void*>(&stage_kernel<N, MODE, MOVING, PREC, 3>)};
  hipError_t e = hipSuccess;
  for (int i = 0; i < 4 && e == hipSuccess; ++i)
    e = hipFuncSetAttribute(fns[i], hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  return e;
}

template <int N, int PREC>
hipError_t stage_prepare_prec(int* blocks_per_cu) {
  hipError_t e = set_lds_limit<N, MODE_RHS, false, PREC>();
  if (e == hipSuccess) e = set_lds_limit<N, MODE_STAGE, false, PREC>();
  if (e == hipSuccess) e = set_lds_limit<N, MODE_RHS, true, PREC>();
  if (e == hipSuccess) e = set_lds_limit<N, MODE_STAGE, true, PREC>();
  if (e != hipSuccess) return e;
  int nb = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &nb, reinterpret_cast<const void*>(&stage_kernel<N, MODE_STAGE, true, PREC, 0>), kThreads,
      Shape<N, PREC>::total * sizeof(float));
  if (e != hipSuccess) return e;
  *blocks_per_cu = std::max(nb, 1);
  return hipSuccess;
}

template <int N>
hipError_t stage_prepare(int precision, int* blocks_per_cu) {
  return precision == 1 ? stage_prepare_prec<N, PREC_BF16>(blocks_per_cu)
                        : stage_prepare_prec<N, PREC_FP32>(blocks_per_cu);
}

template <int N, int MODE, bool MOVING, int PREC>
void stage_launch(int blocks, hipStream_t s, const DeviceMesh& m, const float* q_in, float* q_out,
                  float* res, float* out, float a, float b, double c, double t_host,
                  double dt_host, RunScalars* run, int rate_out) {
  const size_t lds = size_t(Shape<N, PREC>::total) * sizeof(float);
  const int extra = (m.sigma ? EXTRA_DAMP : 0) | (m.curved_flag ? EXTRA_CURVED : 0);
#define DG_STAGE_EXTRA(X)                                                          \
  stage_kernel<N, MODE, MOVING, PREC, X><<<blocks, kThreads, lds, s>>>(            \
      m, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, rate_out)
  switch (extra) {
    case 0: DG_STAGE_EXTRA(0); break;
    case 1: DG_STAGE_EXTRA(1); break;
    case 2: DG_STAGE_EXTRA(2); break;
    default: DG_STAGE_EXTRA(3); break;
  }
#undef DG_STAGE_EXTRA
}

template <int N, int PREC>
void stage_launch_mode(int mode, bool moving, int blocks, hipStream_t s, const DeviceMesh& m,
                       const float* q_in, float* q_out, float* res, float* out, float a, float b,
                       double c, double t_host, double dt_host, RunScalars* run, int rate_out) {
  if (mode == MODE_RHS) {
    if (moving) stage_launch<N, MODE_RHS, true, PREC>(blocks, s, m, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, 0);
    else stage_launch<N, MODE_RHS, false, PREC>(blocks, s, m, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, 0);
  } else {
    if (moving) stage_launch<N, MODE_STAGE, true, PREC>(blocks, s, m, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, rate_out);
    else stage_launch<N, MODE_STAGE, false, PREC>(blocks, s, m, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, rate_out);
  }
}

template <int N>
hipError_t stage_dispatch(const DeviceMesh& m, int mode, const float* q_in, float* q_out,
                          float* res, float* out, float a, float b, double c, double t_host,
                          double dt_host, RunScalars* run, int rate_out, hipStream_t s) {
  const int64_t tiles = (m.K + kTileE - 1) / kTileE;
  const int blocks = int(std::max<int64_t>(1, std::min<int64_t>(tiles, int64_t(m.num_cu) * m.blocks_per_cu)));
  const bool moving = m.phys.u0[0] != 0.0f || m.phys.u0[1] != 0.0f || m.phys.u0[2] != 0.0f;
  const int ro = (run != nullptr && rate_out) ? 1 : 0;
  if (m.precision == 1)
    stage_launch_mode<N, PREC_BF16>(mode, moving, blocks, s, m, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, ro);
  else
    stage_launch_mode<N, PREC_FP32>(mode, moving, blocks, s, m, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, ro);
  return hipGetLastError();
}

template <int N>
hipError_t rate_dispatch(const DeviceMesh& m, const float* q, RunScalars* run, hipStream_t s) {
  using S = Shape<N>;
  const int64_t total = m.K * S::NF;
  const int blocks = int(std::min<int64_t>((total + 255) / 256, 1024));
  rate_kernel<N><<<blocks, 256, 0, s>>>(m, q, run);
  return hipGetLastError();
}

}  // namespace

template <int N>
std::vector<float> pack_operator_n(const double* Dr, const double* Ds, const double* Dt,
                                   const double* LIFT) {
  using S = Shape<N>;
  std::vector<float> A(size_t(S::KT) * S::AS, 0.0f);
  const double* D[3] = {Dr, Ds, Dt};
  for (int k = 0; k < S::KT; ++k)
    for (int mrow = 0; mrow < S::Np; ++mrow) {
      double v = 0.0;
      if (k < S::KV) {
        const int a = k / S::NQP, j = k - a * S::NQP;
        if (j < S::Np) v = -D[a][size_t(mrow) * S::Np + j];
      } else {
        v = LIFT[size_t(mrow) * S::NF + (k - S::KV)];
      }
      A[size_t(k) * S::AS + mrow] = float(v);
    }
  return A;
}

std::vector<float> pack_operator(int N, const double* Dr, const double* Ds, const double* Dt,
                                 const double* LIFT) {
  switch (N) {
    case 1: return pack_operator_n<1>(Dr, Ds, Dt, LIFT);
    case 2: return pack_operator_n<2>(Dr, Ds, Dt, LIFT);
    case 3: return pack_operator_n<3>(Dr, Ds, Dt, LIFT);
    case 4: return pack_operator_n<4>(Dr, Ds, Dt, LIFT);
    case 5: return pack_operator_n<5>(Dr, Ds, Dt, LIFT);
    default: return {};
  }
}

static uint16_t to_bf16_rne(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

static float from_bf16(uint16_t h) {
  const uint32_t u = uint32_t(h) << 16;
  float x;
  std::memcpy(&x, &u, 4);
  return x;
}

template <int N>
std::vector<uint16_t> pack_operator_bf16_n(const double* Dr, const double* Ds, const double* Dt) {
  using S = Shape<N, PREC_BF16>;
  std::vector<uint16_t> A(size_t(2) * S::MP * S::KVB, 0);
  const double* D[3] = {Dr, Ds, Dt};
  for (int mrow = 0; mrow < S::Np; ++mrow)
    for (int kb = 0; kb < S::NKB; ++kb)
      for (int gg = 0; gg < 4; ++gg)
        for (int jj = 0; jj < 2; ++jj)
          for (int a = 0; a < 3; ++a) {
            const int j = 8 * kb + 2 * gg + jj;
            if (j >= S::Np) continue;
            const float x = float(-D[a][size_t(mrow) * S::Np + j]);
            const uint16_t hi = to_bf16_rne(x);
            const uint16_t lo = to_bf16_rne(x - from_bf16(hi));
            const size_t k = size_t(kb) * 32 + 8 * gg + 3 * jj + a;
            A[size_t(mrow) * S::KVB + k] = hi;
            A[(size_t(S::MP) + mrow) * S::KVB + k] = lo;
          }
  return A;
}

std::vector<uint16_t> pack_operator_bf16(int N, const double* Dr, const double* Ds,
                                         const double* Dt) {
  switch (N) {
    case 1: return pack_operator_bf16_n<1>(Dr, Ds, Dt);
    case 2: return pack_operator_bf16_n<2>(Dr, Ds, Dt);
    case 3: return pack_operator_bf16_n<3>(Dr, Ds, Dt);
    case 4: return pack_operator_bf16_n<4>(Dr, Ds, Dt);
    case 5: return pack_operator_bf16_n<5>(Dr, Ds, Dt);
    default: return {};
  }
}

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

hipError_t prepare_kernels(int N, int precision, int* blocks_per_cu) {
  if (spec_stage_supported(N, precision)) {
    const hipError_t e = prepare_spec_stage(N);
    if (e != hipSuccess) return e;
  }
  switch (N) {
    case 1: return stage_prepare<1>(precision, blocks_per_cu);
    case 2: return stage_prepare<2>(precision, blocks_per_cu);
    case 3: return stage_prepare<3>(precision, blocks_per_cu);
    case 4: return stage_prepare<4>(precision, blocks_per_cu);
    case 5: return stage_prepare<5>(precision, blocks_per_cu);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_stage(const DeviceMesh& m, int mode, const float* q_in, float* q_out, float* res,
                        float* out, float a, float b, double c, double t_host, double dt_host,
                        RunScalars* run, int rate_out, hipStream_t s) {
  if (m.variant == 1 && spec_stage_supported(m.N, m.precision))
    return launch_spec_stage(m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run,
                             rate_out, s);
  switch (m.N) {
    case 1: return stage_dispatch<1>(m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, rate_out, s);
    case 2: return stage_dispatch<2>(m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, rate_out, s);
    case 3: return stage_dispatch<3>(m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, rate_out, s);
    case 4: return stage_dispatch<4>(m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, rate_out, s);
    case 5: return stage_dispatch<5>(m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, rate_out, s);
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
  finalize_kernel<<<1, kRateParts, 0, s>>>(run);
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
