// Learned boundary closure: a 78-128-128-75 GELU multilayer perceptron that
// maps a boundary face's interior trace (perturbation, normalized) and its
// unit normal to the exterior trace.  FP32 training kernels (forward with
// saved pre-activations, backward, Adam) on MFMA f32, BF16 inference on MFMA
// bf16 with FP32 accumulation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace dg {

constexpr int kMlpIn = 78, kMlpH = 128, kMlpOut = 75;
constexpr int kMlpNfp = 15;  // face nodes at N = 4
// flat parameter vector: W1 [H][In], b1 [H], W2 [H][H], b2 [H], W3 [Out][H], b3 [Out]
constexpr int kOW1 = 0;
constexpr int kOB1 = kOW1 + kMlpH * kMlpIn;
constexpr int kOW2 = kOB1 + kMlpH;
constexpr int kOB2 = kOW2 + kMlpH * kMlpH;
constexpr int kOW3 = kOB2 + kMlpH;
constexpr int kOB3 = kOW3 + kMlpOut * kMlpH;
constexpr int kMlpParams = kOB3 + kMlpOut;  // 36299

// BF16 weights, rows padded for conflict-free 16-byte LDS reads:
// W1 [128][104] (in 78 -> 96 used), W2 [128][136], W3 [80][136]
constexpr int kS1 = 104, kS2 = 136;
constexpr int kBfW1 = 0;
constexpr int kBfW2 = kBfW1 + 128 * kS1;
constexpr int kBfW3 = kBfW2 + 128 * kS2;
constexpr int kBfTotal = kBfW3 + 80 * kS2;  // bf16 elements

// Training workspace for up to `cap` rows.
struct MlpWork {
  int64_t cap = 0;
  float* x = nullptr;     // [cap][78] gathered minibatch inputs
  float* y = nullptr;     // [cap][75] gathered minibatch targets
  float* z1 = nullptr;    // [cap][128] pre-activations
  float* a1 = nullptr;
  float* z2 = nullptr;
  float* a2 = nullptr;
  float* yh = nullptr;    // [cap][75] output
  float* d3 = nullptr;    // [cap][75] dL/dy
  float* d2 = nullptr;    // [cap][128] dL/dz2
  float* d1 = nullptr;    // [cap][128] dL/dz1
  float* lrow = nullptr;  // [cap] per-row loss
  float* lsum = nullptr;  // [1]
  // [8][128][129] chunk sums of the weight-gradient products (null: those
  // products run unsplit)
  float* part = nullptr;
};
constexpr int64_t kMlpPartFloats = 8 * 128 * 129;

// Fill `grads` (device, kMlpParams) with dL/dparams for rows (X, Y) [B]
// and write the mean loss to *loss_dev.  Deterministic.
hipError_t mlp_grad_f32(const float* P, const float* X, const float* Y, int64_t B, float eps,
                        const MlpWork& w, float* grads, float* loss_dev, hipStream_t s);

// Forward in FP32: Y [B][75] (uses w.z1..a2 as scratch).
hipError_t mlp_forward_f32(const float* P, const float* X, int64_t B, const MlpWork& w,
                           float* Y, hipStream_t s);

// Copies rows idx[i] (clamped to [0, n_rows)) of X and Y into w.x, w.y.
hipError_t mlp_gather_rows(const float* X, const float* Y, const int64_t* idx, int64_t B,
                           int64_t n_rows, const MlpWork& w, hipStream_t s);

// Adam: P -= lr * mhat / (sqrt(vhat) + eps), bias corrections c1 = 1/(1-b1^t), c2 = 1/(1-b2^t).
hipError_t mlp_adam(float* P, const float* g, float* m, float* v, float lr, float b1, float b2,
                    float eps, float c1, float c2, hipStream_t s);

// BF16 copy of the weights in the padded layout above.
hipError_t mlp_pack_bf16(const float* P, uint16_t* Wb, hipStream_t s);

// BF16 inference: Y [B][75] = MLP(X [B][78]).
hipError_t mlp_infer_bf16(const uint16_t* Wb, const float* P, const float* X, int64_t B,
                          float* Y, hipStream_t s);

// Learned ghost traces for the faces of a context tagged learned: for face
// j = (k, f) = lface[j], from the interior trace of q (perturbation
// [K][5][Np]) the characteristic ghost moved by `blend` toward the network's
// exterior trace (its input: that characteristic ghost, scaled), or the characteristic ghost alone when the face's max |p'|
// is outside [plo, phi] or the network state is non-physical; written to
// ghost[j][5][Np] at nodes 0..Nfp-1 (the neighbour layout of the stage
// kernel's gathers).
struct LearnedBC {
  const uint16_t* Wb = nullptr;
  const float* P = nullptr;
  const int32_t* lface = nullptr;  // [nl] k * 4 + f
  int64_t nl = 0;
  float* ghost = nullptr;          // [nl][5][Np]
  float norm = 0.0f;               // input scale: > 0 fixed, else each face's max |q'| of its input
  float plo = 0.0f, phi = 0.0f;    // window of max |p'| where the network is used
  float blend = 1.0f;              // ghost = char + blend * (network - char)
};
hipError_t launch_learned_ghost(const DeviceMesh& m, const LearnedBC& L, const float* q,
                                hipStream_t s);

// Network input rows X [nf][78] (the characteristic ghost of the interior
// trace, then the normal) and, when Y is not null, exterior traces Y [nf][75]
// for faces faces[j] = k * 4 + f of q, both divided by `norm` (> 0) or by the
// largest |q'| of the face's characteristic ghost (norm <= 0).  Interior faces
// take the neighbour trace; boundary faces the ghost of their tag at inflow
// pressure 0.
hipError_t launch_sample_traces(const DeviceMesh& m, const float* q, const int64_t* faces,
                                int64_t nf, float norm, float* X, float* Y, hipStream_t s);

}  // namespace dg
