// Role-specialized fused stage kernel (gfx950 / CDNA4).
//
// Same arithmetic and contract as the tile-cooperative stage kernel: the
// nodal strong form f(q) = -(Dr Fr + Ds Fs + Dt Ft) + LIFT dF (Appendix A,
// Eq. 10) with the local Lax-Friedrichs jump
// dF = Fscale/2 [n.(F- - F+) - lambda (q- - q+)], fused with the low-storage
// RK update (Eq. 12).  One block of eight wavefronts per CU, two roles, and a
// three-deep software pipeline over the block's tiles of 16 elements:
//
//   surface wavefronts (4..7), one per local face f: at iteration i they
//     prefetch tile i+1 (state, FP64 geometry, connectivity, and the
//     exterior traces of face f) into registers, compute tile i's traces,
//     ghost states, face speed lambda (maximum over the face's nodes and both
//     sides, reduced across the four lanes of an element with shuffles) and
//     the jump dF of face f into an LDS buffer in the MFMA operand layout,
//     on the last stage of a step reduce the next time-step rate of tile i-2
//     from its new state, and finally store the prefetched tile into LDS;
//   contraction wavefronts (0..3): wavefront c owns conserved variable c (all
//     row tiles) and row tile c of the energy; it holds its share of the
//     operator A = [-Dr -Ds -Dt | LIFT] in registers for the whole launch,
//     and at iteration i forms tile i-1's contravariant fluxes of its
//     variables straight into MFMA f32 16x16x4 products, adds the LIFT
//     products of the jumps, and writes the fused RK update from the
//     accumulators.
//
// One block barrier per iteration; on each SIMD a surface wavefront's VALU
// work overlaps a contraction wavefront's matrix-core work, every global load
// of a tile is issued before the work of the tile ahead of it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "kernels.hpp"

namespace dg {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kTE = 16;     // elements per tile (MFMA n)
constexpr int kW = 8;       // wavefronts per block: 4 contraction + 4 surface
constexpr int kSlots = 3;   // state tiles in LDS: being filled, surface, contraction

template <int N>
struct XShape {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
  static constexpr int NF = 4 * Nfp;              // face nodes per element
  static constexpr int NNQ = (Np + 3) / 4;        // node quads
  static constexpr int NQP = 4 * NNQ;
  static constexpr int KV = 3 * NQP;              // volume contraction rows
  static constexpr int KT = KV + NF;
  static constexpr int KQ = KT / 4;               // contraction quads
  static constexpr int KQV = KV / 4;
  static constexpr int MP = (Np + 15) / 16 * 16;  // output rows padded to 16
  static constexpr int MT = MP / 16;
  static constexpr int AS = (MP % 32 == 16) ? MP : MP + 16;  // row stride of the packed operator
  static constexpr int ST = 5 * Np;               // floats per element state
  static constexpr int NR = (Nfp + 3) / 4;        // face nodes per surface lane
  static_assert(MT <= 4, "each contraction wavefront takes at most one energy row tile");
  // LDS (floats): tables | slots x (state [16][ST], FP64 vgeo [16][9], sgeo
  // [16][16]) | jumps x2 [5][NF][16] | new states x2 [16][ST] | reduction scratch
  static constexpr int oTab = 0;
  static constexpr int tabFloats = (NF + 96 * Nfp + 15) / 16 * 4;
  static constexpr int qFloats = kTE * ST;
  static constexpr int slotFloats = qFloats + kTE * 25 * 2;
  static constexpr int dFloats = 5 * NF * kTE;
  static constexpr int oSlot = oTab + tabFloats;
  static constexpr int oD = oSlot + kSlots * slotFloats;
  static constexpr int oQn = oD + 2 * dFloats;
  static constexpr int oRed = oQn + 2 * qFloats;
  static constexpr int total = oRed + 2 * kW;
  // register-staged prefetch of one slot: 16-byte chunks
  static constexpr int qChunks = qFloats / 4;
  static constexpr int gChunks = kTE * 25 * 2 / 4;   // 72 vgeo + 128 sgeo
  static constexpr int qRounds = (qChunks + 63) / 64;
  static constexpr int qRoundsPerWave = (qRounds + 3) / 4;
  static_assert(qFloats % 4 == 0, "whole 16-byte chunks");
  static_assert(gChunks <= 256, "one geometry chunk per surface lane");
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

__device__ __forceinline__ floatx4 mfma(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Component V of the flux perturbation along direction n (the same
// expressions as normal_flux).
template <int V, bool MOVING>
__device__ __forceinline__ float flux_var(const Phys& P, const Prim& w, const float n[3]) {
  if (V == 0) return w.mp[0] * n[0] + w.mp[1] * n[1] + w.mp[2] * n[2];
  const float dun = w.du[0] * n[0] + w.du[1] * n[1] + w.du[2] * n[2];
  if (!MOVING) {
    if (V == 4) return dun * (w.E + w.p);
    return w.mp[V - 1] * dun + n[V - 1] * w.pp;
  }
  const float u0n = P.u0[0] * n[0] + P.u0[1] * n[1] + P.u0[2] * n[2];
  if (V == 4) return dun * (w.E + w.p) + u0n * (w.Ep + w.pp);
  return w.m[V - 1] * dun + w.mp[V - 1] * u0n + n[V - 1] * w.pp;
}

// The block's tiles: tile_of(i) for i in [0, n).  Each of the 8 XCDs sweeps a
// contiguous range of tiles (its L2 then holds most neighbour traces).
struct Tiles {
  int64_t first, stride;
  int n;
  __device__ int64_t operator()(int i) const { return first + int64_t(i) * stride; }
};

__device__ __forceinline__ Tiles block_tiles(int64_t K) {
  const int64_t ntiles = (K + kTE - 1) / kTE;
  const int G = gridDim.x, nX = G < 8 ? G : 8;
  const int x = blockIdx.x % nX, jb = blockIdx.x / nX;
  const int Gx = G / nX + (x < G % nX ? 1 : 0);
  const int64_t c0 = ntiles * x / nX, c1 = ntiles * (x + 1) / nX;
  Tiles t;
  t.first = c0 + jb;
  t.stride = Gx;
  t.n = t.first < c1 ? int((c1 - t.first + Gx - 1) / Gx) : 0;
  return t;
}

// ---- contraction wavefront -----------------------------------------------------

template <int N, int MODE, bool MOVING, bool DAMP, int CW>
__device__ __forceinline__ void contraction_role(const DeviceMesh& m, const Tiles& T,
                                                 float* lds, const float* __restrict__ q_in,
                                                 float* __restrict__ q_out, float* __restrict__ res,
                                                 float* __restrict__ out, float a_rk, float b_rk,
                                                 float dt, int rate_out) {
  using S = XShape<N>;
  constexpr int Np = S::Np, ST = S::ST, MT = S::MT, AS = S::AS, NF = S::NF;
  constexpr bool HAS_X = CW < MT;   // also row tile CW of the energy (variable 4)
  const Phys& P = m.phys;
  const int lane = threadIdx.x & 63;
  const int e = lane & 15, g = lane >> 4;

  // this wavefront's share of the operator, A[mt*16 + e][4 kq + g], held in
  // registers for the whole launch
  float aR[S::KQ][MT];
#pragma unroll
  for (int kq = 0; kq < S::KQ; ++kq)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) aR[kq][mt] = m.Aop[(4 * kq + g) * AS + mt * 16 + e];
  __syncthreads();   // prologue: the first tile is in LDS

  const bool want_res = MODE == MODE_STAGE && a_rk != 0.0f;
  for (int it = 0; it <= T.n + 1; ++it) {
    if (it >= 1 && it <= T.n) {
      const int ti = it - 1;
      const int64_t k0 = T(ti) * kTE;
      const int ne = int(min<int64_t>(kTE, m.K - k0));
      // (elements of the curved set are left to the curved pass)
      const bool valid = e < ne && !(m.curved_flag && m.curved_flag[k0 + e]);
      const float* sQ = lds + S::oSlot + (ti % kSlots) * S::slotFloats;
      const double* sV = reinterpret_cast<const double*>(sQ + S::qFloats);   // [16][9]
      const float* sD = lds + S::oD + (ti & 1) * S::dFloats;
      const int64_t ebase = (k0 + e) * ST;

      // residual (and damping rates) of this lane's outputs, in flight during
      // the products; loaded branch-free from a clamped index, so that the
      // loads, the fluxes and the products below form one scheduling region
      const int64_t last = m.K * ST - 1;
      float rold[MT + 1][4], sig[MT + 1][4];
#pragma unroll
      for (int b = 0; b <= MT; ++b) {
        const int V = b < MT ? CW : 4, mt = b < MT ? b : CW;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int node = mt * 16 + 4 * g + r;
          int64_t idx = ebase + V * Np + node;
          idx = idx < last ? idx : last;
          // (no residual is read in right-hand-side mode: res may be null there)
          const float x = MODE == MODE_STAGE ? res[idx] : 0.0f;
          rold[b][r] = want_res ? x : 0.0f;
          int64_t si = (k0 + e) * Np + node;
          si = si < m.K * Np - 1 ? si : m.K * Np - 1;
          sig[b][r] = DAMP ? m.sigma[si] : 0.0f;
        }
      }

      floatx4 acc[MT], accx = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = floatx4{0.f, 0.f, 0.f, 0.f};

      float gm[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) gm[i] = float(sV[e * 9 + i]);

      // volume: contravariant fluxes of node 4 nq + g of element e (a lane
      // past the last node evaluates the last node and contributes zero)
#pragma unroll
      for (int nq = 0; nq < S::NNQ; ++nq) {
        const int j = 4 * nq + g;
        const bool in = j < Np;
        const int jc = in ? j : Np - 1;
        float q[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) q[v] = sQ[e * ST + v * Np + jc];
        Prim wv;
        primitive<MOVING>(P, q, wv);
        float Fm[3], Fx[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float d[3] = {gm[a * 3 + 0], gm[a * 3 + 1], gm[a * 3 + 2]};
          const float fm = flux_var<CW, MOVING>(P, wv, d);
          Fm[a] = in ? fm : 0.0f;
          const float fx = HAS_X ? flux_var<4, MOVING>(P, wv, d) : 0.0f;
          Fx[a] = in ? fx : 0.0f;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int kq = a * S::NNQ + nq;
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) acc[mt] = mfma(aR[kq][mt], Fm[a], acc[mt]);
          if (HAS_X) accx = mfma(aR[kq][HAS_X ? CW : 0], Fx[a], accx);
        }
      }
      // surface: the jumps computed by the surface wavefronts
#pragma unroll
      for (int fq = 0; fq < NF / 4; ++fq) {
        const int kq = S::KQV + fq;
        const float bm = sD[(CW * NF + 4 * fq + g) * kTE + e];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = mfma(aR[kq][mt], bm, acc[mt]);
        if (HAS_X) {
          const float bx = sD[(4 * NF + 4 * fq + g) * kTE + e];
          accx = mfma(aR[kq][HAS_X ? CW : 0], bx, accx);
        }
      }

      // epilogue: lane (g, e) holds nodes mt*16 + 4g + r of element e
      float* sQn = lds + S::oQn + (ti & 1) * S::qFloats;
#pragma unroll
      for (int b = 0; b <= MT; ++b) {
        if (b == MT && !HAS_X) break;
        const int V = b < MT ? CW : 4, mt = b < MT ? b : CW;
        const floatx4 r4 = b < MT ? acc[b < MT ? b : 0] : accx;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int node = mt * 16 + 4 * g + r;
          if (!valid || node >= Np) continue;
          const int64_t idx = ebase + V * Np + node;
          const float qv = sQ[e * ST + V * Np + node];
          float rhs = r4[r];
          if (DAMP) rhs -= sig[b][r] * qv;
          if (MODE == MODE_RHS) {
            out[idx] = rhs;
          } else {
            const float rr = dt * rhs + a_rk * rold[b][r];
            const float qn = qv + b_rk * rr;
            res[idx] = rr;
            q_out[idx] = qn;
            if (rate_out) sQn[e * ST + V * Np + node] = qn;
          }
        }
      }
    }
    __syncthreads();
  }
}

// ---- surface wavefront -----------------------------------------------------------

template <int N, int MODE, bool MOVING>
__device__ __forceinline__ void surface_role(const DeviceMesh& m, const Tiles& T, float* lds,
                                             const float* __restrict__ q_in, float pin,
                                             int rate_out, float& rate_best, unsigned& rate_bad) {
  using S = XShape<N>;
  constexpr int Np = S::Np, Nfp = S::Nfp, ST = S::ST, NF = S::NF, NR = S::NR;
  const Phys& P = m.phys;
  const int lane = threadIdx.x & 63;
  const int e = lane & 15, g = lane >> 4;
  const int f = __builtin_amdgcn_readfirstlane((threadIdx.x >> 6) - 4);   // this wavefront's face
  const int sl = f * 64 + lane;                                         // lane among the four
  const uint8_t* sFm = reinterpret_cast<const uint8_t*>(lds + S::oTab);
  const uint8_t* sNN = sFm + NF;

  // connectivity of face f of this lane's element in tile i
  auto load_conn = [&](int i, int& nb, unsigned& fi) {
    nb = -BC_PASSTHRU;
    fi = 0u;
    if (i < T.n) {
      const int64_t k = T(i) * kTE + e;
      if (k < m.K) {
        nb = m.nbr[k * 4 + f];
        fi = m.finfo[k * 4 + f];
      }
    }
  };
  // exterior traces of face f (neighbour state, or the learned ghost trace)
  auto gather = [&](int i, int nb, unsigned fi, float (&tr)[NR][5]) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int v = 0; v < 5; ++v) tr[r][v] = 0.0f;
    if (i >= T.n || T(i) * kTE + e >= m.K) return;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int ii = g + 4 * r;
      if (ii >= Nfp) continue;
      const float* src = nullptr;
      if (nb >= 0) {
        src = q_in + int64_t(nb) * ST + sNN[((f * 4 + (fi & 3)) * 6 + (fi >> 2)) * Nfp + ii];
      } else if (m.lghost && ((-nb) & 7) == BC_LEARNED) {
        src = m.lghost + int64_t((-nb) >> 3) * ST + ii;
      }
      if (src) {
#pragma unroll
        for (int v = 0; v < 5; ++v) tr[r][v] = src[v * Np];
      }
    }
  };
  // register-staged copy of tile i's state and FP64 geometry
  floatx4 pq[S::qRoundsPerWave], pg;
  int pfull = 1;
  auto fetch_slot = [&](int i) {
    if (i >= T.n) return;
    const int64_t k0 = T(i) * kTE;
    const int ne = int(min<int64_t>(kTE, m.K - k0));
    pfull = ne == kTE;
    const float* qg = q_in + k0 * ST;
#pragma unroll
    for (int jj = 0; jj < S::qRoundsPerWave; ++jj) {
      const int c = (f + 4 * jj) * 64 + lane;
      floatx4 x = {0.f, 0.f, 0.f, 0.f};
      if (c < S::qChunks) {
        if (pfull) {
          x = *reinterpret_cast<const floatx4*>(qg + 4 * c);
        } else {
#pragma unroll
          for (int u = 0; u < 4; ++u) x[u] = (4 * c + u < ne * ST) ? qg[4 * c + u] : 0.0f;
        }
      }
      pq[jj] = x;
    }
    floatx4 y = {0.f, 0.f, 0.f, 0.f};
    if (sl < S::gChunks) {
      // chunk sl: two doubles of vgeo [16][9] (chunks 0..71) or sgeo [16][16]
      const bool isv = sl < 72;
      const int d0 = isv ? 2 * sl : 2 * (sl - 72);
      const double* src = isv ? m.vgeo + k0 * 9 : m.sgeo + k0 * 16;
      const int lim = isv ? ne * 9 : ne * 16;
      double2 dd = {0.0, 0.0};
      if (d0 + 1 < lim) {
        dd = *reinterpret_cast<const double2*>(src + d0);
      } else if (d0 < lim) {
        dd.x = src[d0];
      }
      __builtin_memcpy(&y, &dd, sizeof(y));
    }
    pg = y;
  };
  auto store_slot = [&](int i) {
    if (i >= T.n) return;
    float* sQ = lds + S::oSlot + (i % kSlots) * S::slotFloats;
#pragma unroll
    for (int jj = 0; jj < S::qRoundsPerWave; ++jj) {
      const int c = (f + 4 * jj) * 64 + lane;
      if (c < S::qChunks) *reinterpret_cast<floatx4*>(sQ + 4 * c) = pq[jj];
    }
    if (sl < S::gChunks) *reinterpret_cast<floatx4*>(sQ + S::qFloats + 4 * sl) = pg;
  };

  int nbC, nbN, nbNN;
  unsigned fiC, fiN, fiNN;
  float trC[NR][5], trN[NR][5];
  float fs1 = 0.0f, fs2 = 0.0f;   // Fscale of face f in tiles i-1, i-2

  // prologue: tile 0 in LDS and its traces in registers, connectivity of tile 1
  load_conn(0, nbC, fiC);
  load_conn(1, nbN, fiN);
  fetch_slot(0);
  gather(0, nbC, fiC, trC);
  store_slot(0);
  __syncthreads();

  for (int it = 0; it <= T.n + 1; ++it) {
    // 1. next tile: loads in flight during this tile's work
    fetch_slot(it + 1);
    gather(it + 1, nbN, fiN, trN);
    load_conn(it + 2, nbNN, fiNN);

    // 2. this tile's jumps on face f
    float fs0 = 0.0f;
    if (it < T.n) {
      const int64_t k0 = T(it) * kTE;
      const int ne = int(min<int64_t>(kTE, m.K - k0));
      const bool valid = e < ne;
      const float* sQ = lds + S::oSlot + (it % kSlots) * S::slotFloats;
      const double* sSg = reinterpret_cast<const double*>(sQ + S::qFloats) + kTE * 9;
      float n[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) n[d] = float(sSg[e * 16 + f * 4 + d]);
      fs0 = valid ? float(sSg[e * 16 + f * 4 + 3]) : 0.0f;
      const int nb = valid ? nbC : -BC_PASSTHRU;
      const bool ext = nb >= 0 || (m.lghost && ((-nb) & 7) == BC_LEARNED);
      float fd[NR][5], dq[NR][5];
      float lam = 0.0f;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int ii = g + 4 * r;
        if (ii >= Nfp) {
#pragma unroll
          for (int v = 0; v < 5; ++v) fd[r][v] = dq[r][v] = 0.0f;
          continue;
        }
        const int node = sFm[f * Nfp + ii];
        float qm[5], qp[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) qm[v] = sQ[e * ST + v * Np + node];
        Prim wm;
        primitive<MOVING>(P, qm, wm);
        if (ext) {
#pragma unroll
          for (int v = 0; v < 5; ++v) qp[v] = trC[r][v];
        } else {
          ghost(P, -nb, qm, wm, n, pin, qp);
        }
        Prim wp;
        primitive<MOVING>(P, qp, wp);
        lam = fmaxf(lam, fmaxf(normal_speed<MOVING>(P, wm, n), normal_speed<MOVING>(P, wp, n)));
        float fm[5], fp[5];
        normal_flux<MOVING>(P, wm, n, fm);
        normal_flux<MOVING>(P, wp, n, fp);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          fd[r][v] = fm[v] - fp[v];
          dq[r][v] = qm[v] - qp[v];
        }
      }
      // lambda of the face: maximum over the four lanes of element e
      lam = fmaxf(lam, __shfl_xor(lam, 16));
      lam = fmaxf(lam, __shfl_xor(lam, 32));
      const float hs = 0.5f * fs0;
      float* sD = lds + S::oD + (it & 1) * S::dFloats;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int ii = g + 4 * r;
        if (ii >= Nfp) continue;
#pragma unroll
        for (int v = 0; v < 5; ++v)
          sD[(v * NF + f * Nfp + ii) * kTE + e] = hs * (fd[r][v] - lam * dq[r][v]);
      }
    }

    // 3. next step's time-step rate of tile it-2 from its new state (last
    //    stage of a step): max over face nodes of (N+1)^2/2 Fscale (|u| + c)
    if (MODE == MODE_STAGE && rate_out && it >= 2 && it - 2 < T.n) {
      const int64_t k0 = T(it - 2) * kTE;
      const int ne = int(min<int64_t>(kTE, m.K - k0));
      const float* sQn = lds + S::oQn + (it & 1) * S::qFloats;
      if (e < ne && !(m.curved_flag && m.curved_flag[k0 + e])) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const int ii = g + 4 * r;
          if (ii >= Nfp) continue;
          const int node = sFm[f * Nfp + ii];
          float qq[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) qq[v] = sQn[e * ST + v * Np + node];
          Prim wv;
          primitive<MOVING>(P, qq, wv);
          float sp2 = 0.0f;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const float u = P.u0[d] + wv.du[d];
            sp2 += u * u;
          }
          const float rate = P.half_N1sq * fs2 * (sqrtf(sp2) + sqrtf(P.gamma * wv.p / wv.rho));
          if (!(wv.rho > 0.0f) || !(wv.p > 0.0f) || !(rate == rate)) rate_bad = 1u;
          else rate_best = fmaxf(rate_best, rate);
        }
      }
    }

    // 4. the next tile into its slot (its previous tile was retired by the
    //    contraction wavefronts two iterations ago)
    store_slot(it + 1);
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int v = 0; v < 5; ++v) trC[r][v] = trN[r][v];
    nbC = nbN;
    fiC = fiN;
    nbN = nbNN;
    fiN = fiNN;
    fs2 = fs1;
    fs1 = fs0;
    __syncthreads();
  }
}

template <int N, int MODE, bool MOVING, bool DAMP>
__global__ __launch_bounds__(64 * kW) __attribute__((amdgpu_waves_per_eu(2)))
void spec_stage_kernel(DeviceMesh m, const float* __restrict__ q_in, float* __restrict__ q_out,
                       float* __restrict__ res, float* __restrict__ out, float a_rk, float b_rk,
                       double c_rk, double t_host, double dt_host, RunScalars* run,
                       int rate_out) {
  using S = XShape<N>;
  extern __shared__ float lds[];
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  uint8_t* sFm = reinterpret_cast<uint8_t*>(lds + S::oTab);
  uint8_t* sNN = sFm + S::NF;
  for (int i = tid; i < S::NF; i += 64 * kW) sFm[i] = m.fmask[i];
  for (int i = tid; i < 96 * S::Nfp; i += 64 * kW) sNN[i] = m.nbr_node[i];
  __syncthreads();

  const Tiles T = block_tiles(m.K);
  const double tst = stage_time(c_rk, t_host, dt_host, run);
  const float dt = float(run ? run->dt : dt_host);
  const int ro = (MODE == MODE_STAGE && run != nullptr && rate_out) ? 1 : 0;
  float rate_best = 0.0f;
  unsigned rate_bad = 0u;
  switch (w) {
    case 0: contraction_role<N, MODE, MOVING, DAMP, 0>(m, T, lds, q_in, q_out, res, out, a_rk, b_rk, dt, ro); break;
    case 1: contraction_role<N, MODE, MOVING, DAMP, 1>(m, T, lds, q_in, q_out, res, out, a_rk, b_rk, dt, ro); break;
    case 2: contraction_role<N, MODE, MOVING, DAMP, 2>(m, T, lds, q_in, q_out, res, out, a_rk, b_rk, dt, ro); break;
    case 3: contraction_role<N, MODE, MOVING, DAMP, 3>(m, T, lds, q_in, q_out, res, out, a_rk, b_rk, dt, ro); break;
    default:
      surface_role<N, MODE, MOVING>(m, T, lds, q_in, inflow_pressure(m.phys, tst), ro, rate_best,
                                    rate_bad);
  }

  if (ro) {
    // one atomic per block: wavefront maximum, then across the wavefronts
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      rate_best = fmaxf(rate_best, __shfl_xor(rate_best, off));
      rate_bad |= __shfl_xor(rate_bad, off);
    }
    unsigned* red = reinterpret_cast<unsigned*>(lds + S::oRed);
    if ((tid & 63) == 0) {
      red[2 * w] = __float_as_uint(rate_best);
      red[2 * w + 1] = rate_bad;
    }
    __syncthreads();
    if (tid == 0) {
      float b = 0.0f;
      unsigned bd = 0u;
      for (int ww = 0; ww < kW; ++ww) {
        b = fmaxf(b, __uint_as_float(red[2 * ww]));
        bd |= red[2 * ww + 1];
      }
      atomicMax(&run->rate_bits, __float_as_uint(b));
      if (bd) atomicOr(&run->bad, 1u);
    }
  }
}

template <int N, int MODE, bool MOVING, bool DAMP>
hipError_t set_limit() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&spec_stage_kernel<N, MODE, MOVING, DAMP>),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             int(XShape<N>::total * sizeof(float)));
}

template <int N>
hipError_t prepare_n() {
  hipError_t e = hipSuccess;
  const hipError_t r[8] = {set_limit<N, MODE_RHS, false, false>(), set_limit<N, MODE_RHS, false, true>(),
                           set_limit<N, MODE_RHS, true, false>(), set_limit<N, MODE_RHS, true, true>(),
                           set_limit<N, MODE_STAGE, false, false>(), set_limit<N, MODE_STAGE, false, true>(),
                           set_limit<N, MODE_STAGE, true, false>(), set_limit<N, MODE_STAGE, true, true>()};
  for (hipError_t x : r)
    if (x != hipSuccess) e = x;
  return e;
}

template <int N, int MODE, bool MOVING, bool DAMP>
hipError_t launch_nmd(const DeviceMesh& m, const float* q_in, float* q_out, float* res, float* out,
                      float a, float b, double c, double t_host, double dt_host, RunScalars* run,
                      int rate_out, hipStream_t s) {
  const size_t lds = size_t(XShape<N>::total) * sizeof(float);
  const int64_t tiles = (m.K + kTE - 1) / kTE;
  const int blocks = int(std::max<int64_t>(1, std::min<int64_t>(tiles, m.num_cu)));
  spec_stage_kernel<N, MODE, MOVING, DAMP><<<blocks, 64 * kW, lds, s>>>(
      m, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, rate_out);
  return hipGetLastError();
}

template <int N>
hipError_t launch_n(const DeviceMesh& m, int mode, const float* q_in, float* q_out, float* res,
                    float* out, float a, float b, double c, double t_host, double dt_host,
                    RunScalars* run, int rate_out, hipStream_t s) {
  const bool mv = m.phys.u0[0] != 0.0f || m.phys.u0[1] != 0.0f || m.phys.u0[2] != 0.0f;
  const bool dp = m.sigma != nullptr;
#define DG_SPEC_LAUNCH(MODE_, MV_, DP_) \
  return launch_nmd<N, MODE_, MV_, DP_>(m, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, rate_out, s)
  if (mode == MODE_RHS) {
    if (mv) { if (dp) DG_SPEC_LAUNCH(MODE_RHS, true, true); DG_SPEC_LAUNCH(MODE_RHS, true, false); }
    if (dp) DG_SPEC_LAUNCH(MODE_RHS, false, true);
    DG_SPEC_LAUNCH(MODE_RHS, false, false);
  }
  if (mv) { if (dp) DG_SPEC_LAUNCH(MODE_STAGE, true, true); DG_SPEC_LAUNCH(MODE_STAGE, true, false); }
  if (dp) DG_SPEC_LAUNCH(MODE_STAGE, false, true);
  DG_SPEC_LAUNCH(MODE_STAGE, false, false);
#undef DG_SPEC_LAUNCH
}

}  // namespace

bool spec_stage_supported(int N, int precision) { return precision == 0 && N >= 1 && N <= 4; }

hipError_t prepare_spec_stage(int N) {
  switch (N) {
    case 1: return prepare_n<1>();
    case 2: return prepare_n<2>();
    case 3: return prepare_n<3>();
    case 4: return prepare_n<4>();
    default: return hipSuccess;
  }
}

hipError_t launch_spec_stage(const DeviceMesh& m, int mode, const float* q_in, float* q_out,
                             float* res, float* out, float a, float b, double c, double t_host,
                             double dt_host, RunScalars* run, int rate_out, hipStream_t s) {
  switch (m.N) {
    case 1: return launch_n<1>(m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, rate_out, s);
    case 2: return launch_n<2>(m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, rate_out, s);
    case 3: return launch_n<3>(m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, rate_out, s);
    case 4: return launch_n<4>(m, mode, q_in, q_out, res, out, a, b, c, t_host, dt_host, run, rate_out, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dg
