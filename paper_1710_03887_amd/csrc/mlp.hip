// Learned boundary closure kernels (gfx950): FP32 training on MFMA f32
// 16x16x4, BF16 inference on MFMA bf16 16x16x32, the per-stage learned ghost
// traces and the trace sampler.  Every reduction has a fixed order, so
// results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "mlp.hpp"
#include "physics.hpp"

namespace dg {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) +
         x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }

// ---- FP32 GEMM with split-K over the four wavefronts of a block ------------

enum : int { EP_STORE = 0, EP_BIAS = 1, EP_BIAS_GELU = 2, EP_GELU_GRAD = 3, EP_WGRAD = 4 };

// C (M x N) = sum_k A(m, k) B(k, n) with A(m, k) = A[m sam + k sak] and
// B(k, n) = B[k sbk + n sbn].  Epilogues:
//   EP_STORE      C = AB
//   EP_BIAS       C = AB + bias[n]
//   EP_BIAS_GELU  C = AB + bias[n] (pre-activation), C2 = gelu(C)
//   EP_GELU_GRAD  C = AB * gelu'(Z)   (Z in C's layout)
//   EP_WGRAD      C = AB and C2[m] = sum_k A(m, k) (bias gradient: a column
//                 of ones appended to B)
struct Gemm {
  int M, N, K;
  const float* A;
  int64_t sam, sak;
  const float* B;
  int64_t sbk, sbn;
  float* C;
  int64_t ldc;
  const float* bias;
  float* C2;
  const float* Z;
};

// Epilogue of output (mm, n) with the product sum v (n == N: the bias
// gradient column of EP_WGRAD).
template <int EP>
__device__ __forceinline__ void gemm_store(const Gemm& g, int mm, int n, float v) {
  if (EP == EP_WGRAD) {
    if (n < g.N) g.C[int64_t(mm) * g.ldc + n] = v;
    else if (n == g.N) g.C2[mm] = v;
    return;
  }
  if (n >= g.N) return;
  const int64_t o = int64_t(mm) * g.ldc + n;
  if (EP == EP_BIAS || EP == EP_BIAS_GELU) v += g.bias[n];
  if (EP == EP_GELU_GRAD) v *= gelu_grad(g.Z[o]);
  g.C[o] = v;
  if (EP == EP_BIAS_GELU) g.C2[o] = gelu(v);
}

// One 16 x 16 output tile per block; the contraction range is split into
// gridDim.z chunks (chunk z: k in [z kc, (z+1) kc)), and each chunk over the
// four wavefronts (wavefront w: k-quads w, w+4, ...; 8 quads' loads issued
// ahead of their products).  With one chunk the block applies the epilogue;
// otherwise it writes its sum to part[z][mm][n] and gemm_finish_kernel adds
// the chunks in order.  Every sum has a fixed order: results are bitwise
// reproducible.
template <int EP>
__global__ __launch_bounds__(256) void gemm_kernel(Gemm g, int kc, float* part, int ldp) {
  __shared__ floatx4 red[4][64];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, e = lane & 15, q4 = lane >> 4;
  const int m0 = blockIdx.x * 16, n0 = blockIdx.y * 16;
  const int m = m0 + e, n = n0 + e;
  const int kb = blockIdx.z * kc, ke = min(g.K, kb + kc);
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k00 = kb + 4 * w; k00 < ke; k00 += 16 * 8) {
    float a[8], b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = k00 + 16 * u + q4;
      const bool kin = k < ke;
      a[u] = (kin && m < g.M) ? g.A[int64_t(m) * g.sam + int64_t(k) * g.sak] : 0.0f;
      b[u] = 0.0f;
      if (kin) {
        if (EP == EP_WGRAD && n == g.N) b[u] = 1.0f;
        else if (n < g.N) b[u] = g.B[int64_t(k) * g.sbk + int64_t(n) * g.sbn];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], b[u], acc, 0, 0, 0);
  }
  red[w][lane] = acc;
  __syncthreads();
  if (w != 0) return;
  const floatx4 sum = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
  const int ncol = EP == EP_WGRAD ? g.N + 1 : g.N;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int mm = m0 + 4 * q4 + r;
    if (mm >= g.M || n >= ncol) continue;
    if (gridDim.z == 1) gemm_store<EP>(g, mm, n, sum[r]);
    else part[(int64_t(blockIdx.z) * g.M + mm) * ldp + n] = sum[r];
  }
}

// Adds the chunk sums part[0..kz)[mm][n] in order and applies the epilogue.
template <int EP>
__global__ __launch_bounds__(256) void gemm_finish_kernel(Gemm g, int kz, const float* part, int ldp) {
  const int ncol = EP == EP_WGRAD ? g.N + 1 : g.N;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(g.M) * ncol) return;
  const int mm = int(i / ncol), n = int(i % ncol);
  float v = 0.0f;
  for (int z = 0; z < kz; ++z) v += part[(int64_t(z) * g.M + mm) * ldp + n];
  gemm_store<EP>(g, mm, n, v);
}

// Contractions longer than kGemmSplitK are split into chunks of at least
// that length, at most kGemmMaxChunks of them (partial sums in `part`,
// kGemmMaxChunks x 128 x 129 floats).
constexpr int kGemmSplitK = 512, kGemmMaxChunks = 8, kGemmPartLd = kMlpH + 1;
static_assert(kMlpPartFloats >= int64_t(kGemmMaxChunks) * kMlpH * kGemmPartLd,
              "chunk sums must fit the workspace");

template <int EP>
hipError_t gemm(const Gemm& g, hipStream_t s, float* part = nullptr) {
  const int ncol = EP == EP_WGRAD ? g.N + 1 : g.N;
  int kz = 1;
  if (part && g.K > kGemmSplitK && g.M <= kMlpH && ncol <= kGemmPartLd)
    kz = std::min(kGemmMaxChunks, (g.K + kGemmSplitK - 1) / kGemmSplitK);
  const int kc = kz == 1 ? g.K : ((g.K + kz - 1) / kz + 15) / 16 * 16;
  dim3 grid((g.M + 15) / 16, (ncol + 15) / 16, kz);
  gemm_kernel<EP><<<grid, 256, 0, s>>>(g, kc, part, kGemmPartLd);
  if (kz > 1) {
    const int64_t n = int64_t(g.M) * ncol;
    gemm_finish_kernel<EP><<<int((n + 255) / 256), 256, 0, s>>>(g, kz, part, kGemmPartLd);
  }
  return hipGetLastError();
}

Gemm make(int M, int N, int K, const float* A, int64_t sam, int64_t sak, const float* B,
          int64_t sbk, int64_t sbn, float* C, int64_t ldc) {
  Gemm g;
  g.M = M;
  g.N = N;
  g.K = K;
  g.A = A;
  g.sam = sam;
  g.sak = sak;
  g.B = B;
  g.sbk = sbk;
  g.sbn = sbn;
  g.C = C;
  g.ldc = ldc;
  g.bias = nullptr;
  g.C2 = nullptr;
  g.Z = nullptr;
  return g;
}

// ---- loss, reductions, optimizer, data movement ---------------------------

// one wavefront per row: relative squared error and dL/dy_hat
__global__ __launch_bounds__(256) void loss_kernel(const float* yh, const float* y, int64_t B,
                                                   float eps, float* d3, float* lrow) {
  const int lane = threadIdx.x & 63;
  const int64_t row = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (row >= B) return;
  const float* a = yh + row * kMlpOut;
  const float* t = y + row * kMlpOut;
  float num = 0.0f, den = 0.0f;
  for (int j = lane; j < kMlpOut; j += 64) {
    const float r = a[j] - t[j];
    num += r * r;
    den += t[j] * t[j];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    num += __shfl_xor(num, o);
    den += __shfl_xor(den, o);
  }
  den += eps;
  if (lane == 0) lrow[row] = num / den;
  const float sc = 2.0f / (den * float(B));
  for (int j = lane; j < kMlpOut; j += 64) d3[row * kMlpOut + j] = sc * (a[j] - t[j]);
}

// out[0] = scale * sum(x[0..n)), one block, fixed order
__global__ __launch_bounds__(256) void sum_kernel(const float* x, int64_t n, float scale,
                                                  float* out) {
  __shared__ float part[256];
  float acc = 0.0f;
  for (int64_t i = threadIdx.x; i < n; i += 256) acc += x[i];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = part[0] * scale;
}

__global__ void adam_kernel(float* P, const float* g, float* m, float* v, int n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  P[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

__global__ void gather_rows_kernel(const float* X, const float* Y, const int64_t* idx, int64_t B,
                                   int64_t n_rows, float* xo, float* yo) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t row = t / 128;
  const int c = int(t % 128);
  if (row >= B) return;
  const int64_t src = min(max(idx[row], int64_t(0)), n_rows - 1);  // rows outside the set are clamped
  if (c < kMlpIn) xo[row * kMlpIn + c] = X[src * kMlpIn + c];
  if (c < kMlpOut) yo[row * kMlpOut + c] = Y[src * kMlpOut + c];
}

__global__ void pack_bf16_kernel(const float* P, __bf16* Wb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kBfTotal) return;
  float v = 0.0f;
  if (i < kBfW2) {
    const int r = i / kS1, c = i % kS1;
    if (c < kMlpIn) v = P[kOW1 + r * kMlpIn + c];
  } else if (i < kBfW3) {
    const int r = (i - kBfW2) / kS2, c = (i - kBfW2) % kS2;
    if (c < kMlpH) v = P[kOW2 + r * kMlpH + c];
  } else {
    const int r = (i - kBfW3) / kS2, c = (i - kBfW3) % kS2;
    if (r < kMlpOut && c < kMlpH) v = P[kOW3 + r * kMlpH + c];
  }
  Wb[i] = to_bf16(v);
}

// ---- BF16 inference core ----------------------------------------------------

// Per wavefront LDS: sX [16][kS1] inputs, sH1/sH2 [16][kS2] hidden
// activations (bf16); outputs as FP32 [16][80] over sX..sH1 once layer 2 is
// done.
constexpr int kWaveBytes = 16 * kS1 * 2 + 2 * 16 * kS2 * 2;
constexpr int kWeightBytes = kBfTotal * 2;
constexpr int kInferLds = kWeightBytes + 4 * kWaveBytes;
static_assert(16 * 80 * 4 <= 16 * kS1 * 2 + 16 * kS2 * 2, "output tile must fit over sX, sH1");

__device__ __forceinline__ void load_weights(const uint16_t* Wb, uint16_t* sW) {
  const uint4* src = reinterpret_cast<const uint4*>(Wb);
  uint4* dst = reinterpret_cast<uint4*>(sW);
  for (int i = threadIdx.x; i < kWeightBytes / 16; i += blockDim.x) dst[i] = src[i];
}

// one layer: out[face][j] for 16 faces, j over mt tiles; A = W rows (LDS),
// B = activations [face][k] (LDS)
template <int MT, int KB, int SW, int SA>
__device__ __forceinline__ void layer_bf16(const __bf16* W, const __bf16* act, floatx4 (&acc)[MT],
                                           int e, int q4) {
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) acc[mt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    const bf16x8 b = *reinterpret_cast<const bf16x8*>(act + e * SA + kb * 32 + 8 * q4);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(W + (mt * 16 + e) * SW + kb * 32 + 8 * q4);
      acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[mt], 0, 0, 0);
    }
  }
}

// Runs the network on the wavefront's 16 rows in sX; leaves the FP32 outputs
// in sY [16][80] (normalized units).
__device__ __forceinline__ void mlp_wave(const __bf16* sW, const float* P, __bf16* sX,
                                         __bf16* sH1, __bf16* sH2, float* sY) {
  const int lane = threadIdx.x & 63, e = lane & 15, q4 = lane >> 4;
  {
    floatx4 acc[8];
    layer_bf16<8, 3, kS1, kS1>(sW + kBfW1, sX, acc, e, q4);
#pragma unroll
    for (int mt = 0; mt < 8; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = mt * 16 + 4 * q4 + r;
        sH1[e * kS2 + j] = to_bf16(gelu(acc[mt][r] + P[kOB1 + j]));
      }
  }
  __syncthreads();
  {
    floatx4 acc[8];
    layer_bf16<8, 4, kS2, kS2>(sW + kBfW2, sH1, acc, e, q4);
#pragma unroll
    for (int mt = 0; mt < 8; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = mt * 16 + 4 * q4 + r;
        sH2[e * kS2 + j] = to_bf16(gelu(acc[mt][r] + P[kOB2 + j]));
      }
  }
  __syncthreads();
  {
    floatx4 acc[5];
    layer_bf16<5, 4, kS2, kS2>(sW + kBfW3, sH2, acc, e, q4);
#pragma unroll
    for (int mt = 0; mt < 5; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = mt * 16 + 4 * q4 + r;
        sY[e * 80 + j] = j < kMlpOut ? acc[mt][r] + P[kOB3 + j] : 0.0f;
      }
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void infer_kernel(const uint16_t* Wb, const float* P,
                                                    const float* X, int64_t B, float* Y) {
  extern __shared__ uint4 smem4[];
  uint16_t* smem = reinterpret_cast<uint16_t*>(smem4);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __bf16* sW = reinterpret_cast<__bf16*>(smem);
  char* wb = reinterpret_cast<char*>(smem) + kWeightBytes + w * kWaveBytes;
  __bf16* sX = reinterpret_cast<__bf16*>(wb);
  __bf16* sH1 = sX + 16 * kS1;
  __bf16* sH2 = sH1 + 16 * kS2;
  float* sY = reinterpret_cast<float*>(wb);
  load_weights(Wb, smem);
  const int64_t r0 = (int64_t(blockIdx.x) * 4 + w) * 16;
  for (int i = lane; i < 16 * kS1; i += 64) {
    const int row = i / kS1, c = i % kS1;
    const float v = (c < kMlpIn && r0 + row < B) ? X[(r0 + row) * kMlpIn + c] : 0.0f;
    sX[i] = to_bf16(v);
  }
  __syncthreads();
  mlp_wave(sW, P, sX, sH1, sH2, sY);
  for (int i = lane; i < 16 * kMlpOut; i += 64) {
    const int row = i / kMlpOut, j = i % kMlpOut;
    if (r0 + row < B) Y[(r0 + row) * kMlpOut + j] = sY[row * 80 + j];
  }
}

// ---- learned ghost traces (N = 4) -------------------------------------------

constexpr int kNp4 = 35, kNfp4 = 15;
constexpr int kGhostFaces = 16;  // faces per block: the N side of one MFMA tile

// A operand of a weight tile: rows row0 + e, k-block kb (BF16, padded layout)
__device__ __forceinline__ bf16x8 wfrag(const uint16_t* W, int row, int stride, int kb, int q4) {
  return *reinterpret_cast<const bf16x8*>(W + row * stride + kb * 32 + 8 * q4);
}

// One block of four wavefronts per 16 learned faces.  Thread t < 240 owns
// node t % 15 of face t / 15 from the gather to the store and keeps its
// characteristic ghost in registers; the network's output rows are split
// over the wavefronts (wavefront w: hidden tiles 2w, 2w+1 of layers 1 and 2,
// output tiles w and, for w = 0, 4 of layer 3), whose weights each
// wavefront loads from global memory straight into registers at entry, so
// the weights are read once per block and never staged in LDS.
__global__ __launch_bounds__(256) void learned_ghost_kernel(DeviceMesh m, LearnedBC L,
                                                            const float* q) {
  __shared__ __attribute__((aligned(16))) __bf16 sX[kGhostFaces * kS1];
  __shared__ __attribute__((aligned(16))) __bf16 sH1[kGhostFaces * kS2];
  __shared__ __attribute__((aligned(16))) __bf16 sH2[kGhostFaces * kS2];
  // the characteristic ghost [16][75] until the inputs are built, then the
  // network's FP32 outputs [16][80]
  __shared__ float sY[kGhostFaces * 80];
  __shared__ float sNrm[kGhostFaces][3];
  __shared__ float sPmax[kGhostFaces], sScale[kGhostFaces];
  __shared__ unsigned sBad[kGhostFaces];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63, e = lane & 15, q4 = lane >> 4;
  const Phys& P = m.phys;
  const int64_t j0 = int64_t(blockIdx.x) * kGhostFaces;

  // this wavefront's weight and bias fragments (uniform branch on w for the
  // fifth output tile)
  const bool tile4 = w == 0;
  bf16x8 a1[2][3], a2[2][4], a3[2][4];
  float b1[2][4], b2[2][4], b3[2][4];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int h = (2 * w + u) * 16;
#pragma unroll
    for (int kb = 0; kb < 3; ++kb) a1[u][kb] = wfrag(L.Wb + kBfW1, h + e, kS1, kb, q4);
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) a2[u][kb] = wfrag(L.Wb + kBfW2, h + e, kS2, kb, q4);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      b1[u][r] = L.P[kOB1 + h + 4 * q4 + r];
      b2[u][r] = L.P[kOB2 + h + 4 * q4 + r];
    }
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int o = (u == 0 ? w : 4) * 16;
    if (u == 0 || tile4) {
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) a3[u][kb] = wfrag(L.Wb + kBfW3, o + e, kS2, kb, q4);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int jj = o + 4 * q4 + r;
        b3[u][r] = jj < kMlpOut ? L.P[kOB3 + jj] : 0.0f;
      }
    }
  }

  if (t < kGhostFaces) {
    sPmax[t] = 0.0f;
    sScale[t] = 0.0f;
    sBad[t] = 0u;
  }
  __syncthreads();
  // per owned node: the characteristic ghost (the network's input: the
  // interior trace with its incoming acoustic characteristic removed); per
  // face: max |p'| of the interior trace and the ghost's largest |q'|
  const int row = t / kNfp4, ii = t % kNfp4;
  const int64_t j = j0 + row;
  const bool own = t < kGhostFaces * kNfp4 && j < L.nl;
  float qc[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  if (own) {
    const int kf = L.lface[j];
    const int64_t k = kf >> 2;
    const int f = kf & 3;
    const int node = m.fmask[f * kNfp4 + ii];
    const float n[3] = {float(m.sgeo[k * 16 + f * 4 + 0]), float(m.sgeo[k * 16 + f * 4 + 1]),
                        float(m.sgeo[k * 16 + f * 4 + 2])};
    float qm[5], big = 0.0f;
#pragma unroll
    for (int v = 0; v < 5; ++v) qm[v] = q[(k * 5 + v) * kNp4 + node];
    Prim wm;
    primitive<true>(P, qm, wm);
    ghost(P, BC_OUTFLOW_CHAR, qm, wm, n, 0.0f, qc);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      sY[row * kMlpOut + v * kNfp4 + ii] = qc[v];
      big = fmaxf(big, fabsf(qc[v]));
    }
    if (ii < 3) sNrm[row][ii] = n[ii];
    atomicMax(reinterpret_cast<unsigned*>(&sPmax[row]), __float_as_uint(fabsf(wm.pp)));
    atomicMax(reinterpret_cast<unsigned*>(&sScale[row]), __float_as_uint(big));
  }
  __syncthreads();
  if (t < kGhostFaces && L.norm > 0.0f) sScale[t] = L.norm;
  __syncthreads();
  // inputs: characteristic ghost / scale (variable-major), then the normal
  for (int i = t; i < kGhostFaces * kS1; i += 256) {
    const int r = i / kS1, c = i % kS1;
    float v = 0.0f;
    if (j0 + r < L.nl && c < kMlpIn) {
      if (c < 5 * kNfp4) {
        const float sc = sScale[r];
        v = sc > 0.0f ? sY[r * kMlpOut + c] / sc : 0.0f;
      } else {
        v = sNrm[r][c - 5 * kNfp4];
      }
    }
    sX[i] = to_bf16(v);
  }
  __syncthreads();
  // layer 1: hidden tiles 2w, 2w+1
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 3; ++kb) {
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(sX + e * kS1 + kb * 32 + 8 * q4);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[u][kb], b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
      sH1[e * kS2 + (2 * w + u) * 16 + 4 * q4 + r] = to_bf16(gelu(acc[r] + b1[u][r]));
  }
  __syncthreads();
  // layer 2
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(sH1 + e * kS2 + kb * 32 + 8 * q4);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[u][kb], b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
      sH2[e * kS2 + (2 * w + u) * 16 + 4 * q4 + r] = to_bf16(gelu(acc[r] + b2[u][r]));
  }
  __syncthreads();
  // layer 3: output tiles w and (w = 0) 4, FP32 over sY
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    if (u == 1 && !tile4) break;
    const int o = (u == 0 ? w : 4) * 16;
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(sH2 + e * kS2 + kb * 32 + 8 * q4);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3[u][kb], b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) sY[e * 80 + o + 4 * q4 + r] = acc[r] + b3[u][r];
  }
  __syncthreads();
  // learned ghost = characteristic ghost + blend * (scale * network output -
  // characteristic ghost), with a physical check at every node
  float qg[5];
  if (own) {
    const float sc = sScale[row];
#pragma unroll
    for (int v = 0; v < 5; ++v) qg[v] = qc[v] + L.blend * (sc * sY[row * 80 + v * kNfp4 + ii] - qc[v]);
    Prim wg;
    primitive<true>(P, qg, wg);
    if (!(wg.rho > 0.0f) || !(wg.p > 0.0f) || !(sc > 0.0f)) atomicOr(&sBad[row], 1u);
  }
  __syncthreads();
  if (own) {
    const float pm = sPmax[row];
    const bool use = !sBad[row] && pm >= L.plo && pm <= L.phi;
#pragma unroll
    for (int v = 0; v < 5; ++v) L.ghost[(j * 5 + v) * kNp4 + ii] = use ? qg[v] : qc[v];
  }
}

// ---- trace sampler ------------------------------------------------------------

// one wavefront per face, lane = face node
template <int N>
__global__ __launch_bounds__(256) void sample_kernel(DeviceMesh m, const float* q,
                                                     const int64_t* faces, int64_t nf, float norm,
                                                     float* X, float* Y) {
  constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6, Nfp = (N + 1) * (N + 2) / 2;
  static_assert(Nfp <= 64, "one wavefront per face");
  const int ii = threadIdx.x & 63;
  const int64_t j = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (j >= nf) return;
  const int64_t kf = faces[j];
  const int64_t k = kf >> 2;
  const int f = int(kf & 3);
  if (kf < 0 || k >= m.K) return;  // not a face of this mesh
  const bool node_lane = ii < Nfp;
  float qm[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, qp[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  float n[3] = {float(m.sgeo[k * 16 + f * 4 + 0]), float(m.sgeo[k * 16 + f * 4 + 1]),
                float(m.sgeo[k * 16 + f * 4 + 2])};
  float big = 0.0f, qc[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  if (node_lane) {
    const int node = m.fmask[f * Nfp + ii];
#pragma unroll
    for (int v = 0; v < 5; ++v) qm[v] = q[(k * 5 + v) * Np + node];
    Prim wm;
    primitive<true>(m.phys, qm, wm);
    ghost(m.phys, BC_OUTFLOW_CHAR, qm, wm, n, 0.0f, qc);
#pragma unroll
    for (int v = 0; v < 5; ++v) big = fmaxf(big, fabsf(qc[v]));
    const int nb = m.nbr[k * 4 + f];
    if (nb >= 0) {
      const int inf = m.finfo[k * 4 + f];
      const int n2 = m.nbr_node[((f * 4 + (inf & 3)) * 6 + (inf >> 2)) * Nfp + ii];
#pragma unroll
      for (int v = 0; v < 5; ++v) qp[v] = q[(int64_t(nb) * 5 + v) * Np + n2];
    } else {
      ghost(m.phys, (-nb) & 7, qm, wm, n, 0.0f, qp);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) big = fmaxf(big, __shfl_xor(big, o));
  const float sc = norm > 0.0f ? norm : big;
  const float inv = sc > 0.0f ? 1.0f / sc : 0.0f;
  const int in = 5 * Nfp + 3, out = 5 * Nfp;
  if (node_lane) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      X[j * in + v * Nfp + ii] = qc[v] * inv;
      if (Y) Y[j * out + v * Nfp + ii] = qp[v] * inv;
    }
  }
  if (ii < 3) X[j * in + 5 * Nfp + ii] = n[ii];
}

}  // namespace

// ---- host entry points ----------------------------------------------------------

hipError_t mlp_forward_f32(const float* P, const float* X, int64_t B, const MlpWork& w, float* Y,
                           hipStream_t s) {
  const int b = int(B);
  Gemm g1 = make(b, kMlpH, kMlpIn, X, kMlpIn, 1, P + kOW1, 1, kMlpIn, w.z1, kMlpH);
  g1.bias = P + kOB1;
  g1.C2 = w.a1;
  hipError_t e = gemm<EP_BIAS_GELU>(g1, s);
  Gemm g2 = make(b, kMlpH, kMlpH, w.a1, kMlpH, 1, P + kOW2, 1, kMlpH, w.z2, kMlpH);
  g2.bias = P + kOB2;
  g2.C2 = w.a2;
  if (e == hipSuccess) e = gemm<EP_BIAS_GELU>(g2, s);
  Gemm g3 = make(b, kMlpOut, kMlpH, w.a2, kMlpH, 1, P + kOW3, 1, kMlpH, Y, kMlpOut);
  g3.bias = P + kOB3;
  if (e == hipSuccess) e = gemm<EP_BIAS>(g3, s);
  return e;
}

hipError_t mlp_grad_f32(const float* P, const float* X, const float* Y, int64_t B, float eps,
                        const MlpWork& w, float* grads, float* loss_dev, hipStream_t s) {
  const int b = int(B);
  hipError_t e = mlp_forward_f32(P, X, B, w, w.yh, s);
  if (e != hipSuccess) return e;
  loss_kernel<<<int((B + 3) / 4), 256, 0, s>>>(w.yh, Y, B, eps, w.d3, w.lrow);
  sum_kernel<<<1, 256, 0, s>>>(w.lrow, B, 1.0f / float(B), loss_dev);
  // layer 3: dW3 = d3^T a2, db3 = sum d3; d2 = (d3 W3) * gelu'(z2)
  Gemm w3 = make(kMlpOut, kMlpH, b, w.d3, 1, kMlpOut, w.a2, kMlpH, 1, grads + kOW3, kMlpH);
  w3.C2 = grads + kOB3;
  e = gemm<EP_WGRAD>(w3, s, w.part);
  Gemm d2 = make(b, kMlpH, kMlpOut, w.d3, kMlpOut, 1, P + kOW3, kMlpH, 1, w.d2, kMlpH);
  d2.Z = w.z2;
  if (e == hipSuccess) e = gemm<EP_GELU_GRAD>(d2, s);
  // layer 2
  Gemm w2 = make(kMlpH, kMlpH, b, w.d2, 1, kMlpH, w.a1, kMlpH, 1, grads + kOW2, kMlpH);
  w2.C2 = grads + kOB2;
  if (e == hipSuccess) e = gemm<EP_WGRAD>(w2, s, w.part);
  Gemm d1 = make(b, kMlpH, kMlpH, w.d2, kMlpH, 1, P + kOW2, kMlpH, 1, w.d1, kMlpH);
  d1.Z = w.z1;
  if (e == hipSuccess) e = gemm<EP_GELU_GRAD>(d1, s);
  // layer 1
  Gemm w1 = make(kMlpH, kMlpIn, b, w.d1, 1, kMlpH, X, kMlpIn, 1, grads + kOW1, kMlpIn);
  w1.C2 = grads + kOB1;
  if (e == hipSuccess) e = gemm<EP_WGRAD>(w1, s, w.part);
  if (e == hipSuccess) e = hipGetLastError();
  return e;
}

hipError_t mlp_gather_rows(const float* X, const float* Y, const int64_t* idx, int64_t B,
                           int64_t n_rows, const MlpWork& w, hipStream_t s) {
  const int64_t n = B * 128;
  gather_rows_kernel<<<int((n + 255) / 256), 256, 0, s>>>(X, Y, idx, B, n_rows, w.x, w.y);
  return hipGetLastError();
}

hipError_t mlp_adam(float* P, const float* g, float* m, float* v, float lr, float b1, float b2,
                    float eps, float c1, float c2, hipStream_t s) {
  adam_kernel<<<(kMlpParams + 255) / 256, 256, 0, s>>>(P, g, m, v, kMlpParams, lr, b1, b2, eps,
                                                        c1, c2);
  return hipGetLastError();
}

hipError_t mlp_pack_bf16(const float* P, uint16_t* Wb, hipStream_t s) {
  pack_bf16_kernel<<<(kBfTotal + 255) / 256, 256, 0, s>>>(P, reinterpret_cast<__bf16*>(Wb));
  return hipGetLastError();
}

static hipError_t lds_attr(const void* fn) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kInferLds);
}

hipError_t mlp_infer_bf16(const uint16_t* Wb, const float* P, const float* X, int64_t B, float* Y,
                          hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipError_t e = lds_attr(reinterpret_cast<const void*>(&infer_kernel));
  if (e != hipSuccess) return e;
  infer_kernel<<<int((B + 63) / 64), 256, kInferLds, s>>>(Wb, P, X, B, Y);
  return hipGetLastError();
}

hipError_t launch_learned_ghost(const DeviceMesh& m, const LearnedBC& L, const float* q,
                                hipStream_t s) {
  if (L.nl <= 0) return hipSuccess;
  if (m.N != 4) return hipErrorInvalidValue;
  learned_ghost_kernel<<<int((L.nl + kGhostFaces - 1) / kGhostFaces), 256, 0, s>>>(m, L, q);
  return hipGetLastError();
}

hipError_t launch_sample_traces(const DeviceMesh& m, const float* q, const int64_t* faces,
                                int64_t nf, float norm, float* X, float* Y, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  const int blocks = int((nf + 3) / 4);
  switch (m.N) {
    case 1: sample_kernel<1><<<blocks, 256, 0, s>>>(m, q, faces, nf, norm, X, Y); break;
    case 2: sample_kernel<2><<<blocks, 256, 0, s>>>(m, q, faces, nf, norm, X, Y); break;
    case 3: sample_kernel<3><<<blocks, 256, 0, s>>>(m, q, faces, nf, norm, X, Y); break;
    case 4: sample_kernel<4><<<blocks, 256, 0, s>>>(m, q, faces, nf, norm, X, Y); break;
    case 5: sample_kernel<5><<<blocks, 256, 0, s>>>(m, q, faces, nf, norm, X, Y); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace dg
