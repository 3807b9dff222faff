// Launch interface between the C ABI and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "physics.hpp"

namespace dg {

// Everything a stage kernel reads, as device pointers.
struct DeviceMesh {
  int N = 0, Np = 0, Nfp = 0;
  int64_t K = 0;
  int precision = 0;
  int num_cu = 256;          // compute units of the device
  int blocks_per_cu = 1;     // resident stage blocks per CU
  const float* Aop = nullptr;       // contraction operator, layout from pack_operator
  const uint16_t* Abf = nullptr;    // split-BF16 volume operator, layout from pack_operator_bf16
  const uint8_t* fmask = nullptr;   // [4][Nfp]
  const uint8_t* nbr_node = nullptr;  // [4][4][6][Nfp]
  const double* vgeo = nullptr;     // [K][9]   d(r,s,t)/d(x,y,z)
  const double* sgeo = nullptr;     // [K][4][4] nx ny nz Fscale
  // the same geometry in FP32 for the tile-cooperative stage kernel, per
  // tile of 16 elements component-major: [tiles][25][16] (the 9 metric
  // terms, then nx, ny, nz, Fscale of faces 0..3), zero past element K - 1
  const float* geo32 = nullptr;
  const int32_t* nbr = nullptr;     // [K][4] neighbour element, or -tag
  const uint8_t* finfo = nullptr;   // [K][4] neighbour face | orientation << 2
  // learned ghost traces [n_learned][5][Np] (nodes 0..Nfp-1), or null; a
  // learned face's nbr entry is -(BC_LEARNED + 8 * its index)
  const float* lghost = nullptr;
  // absorbing layer: damping rate per node [K][Np] (rhs -= sigma q'), or null
  const float* sigma = nullptr;
  // [K] 1 for the elements of the curved set, or null: the stage kernels
  // leave their outputs and their share of the time-step rate to the curved
  // pass
  const uint8_t* curved_flag = nullptr;
  int variant = 0;                  // stage kernel: 0 tile-cooperative, 1 role-specialized
  // 0: nodal strong form + LSERK4; 1: weak form with Gauss quadrature + RK2
  int scheme = 0;
  const float* qtab = nullptr;      // quadrature-scheme tables (scheme 1)
  Phys phys;
};

// Slots over which passes with many small blocks spread their time-step
// rate maxima (one word would queue their atomics); the finalize kernel
// folds them in.
constexpr int kRateParts = 256;
static_assert(kRateParts % 64 == 0 && (kRateParts & (kRateParts - 1)) == 0,
              "whole wavefronts, and a mask picks the slot");

// Device scalars of a run: time, step, CFL reduction and error flags.
struct RunScalars {
  double t;
  double dt;
  double cfl;
  double fixed_dt;   // > 0: every step takes this dt instead of the CFL rule
  int64_t step;
  int64_t first_bad;
  uint32_t rate_bits;
  uint32_t bad;
  uint32_t rate_part[kRateParts];   // more rate maxima (ordered float bits), 0 when unused
};

enum StageMode : int { MODE_RHS = 0, MODE_STAGE = 1 };

// One right-hand-side evaluation (MODE_RHS: out = f(q_in)) or one fused
// low-storage RK stage (MODE_STAGE: res = a res + dt f(q_in);
// q_out = q_in + b res).  Time is t_host + c dt_host, or read from
// run->t/run->dt when `run` is not null.  With run and rate_out set (last
// stage of a step), the stage also reduces the next step's time-step rate
// from q_out into run->rate_bits and flags non-physical states.
hipError_t launch_stage(const DeviceMesh& m, int mode, const float* q_in, float* q_out,
                        float* res, float* out, float a, float b, double c, double t_host,
                        double dt_host, RunScalars* run, int rate_out, hipStream_t s);

// The role-specialized stage kernel (same contract as launch_stage): four
// surface and four contraction wavefronts per block, one block per CU; FP32
// form at N <= 4.  prepare_spec_stage raises its dynamic-LDS limit.
bool spec_stage_supported(int N, int precision);
hipError_t prepare_spec_stage(int N);
hipError_t launch_spec_stage(const DeviceMesh& m, int mode, const float* q_in, float* q_out,
                             float* res, float* out, float a, float b, double c, double t_host,
                             double dt_host, RunScalars* run, int rate_out, hipStream_t s);

// Max of (N+1)^2/2 Fscale (|u|+c) over interior face traces into
// run->rate_bits (as ordered float bits); flags non-physical traces.
hipError_t launch_rate(const DeviceMesh& m, const float* q, RunScalars* run, hipStream_t s);

// dt = cfl / rate (the maximum of rate_bits and rate_part); records the first
// non-physical step; clears the reduction.
hipError_t launch_finalize(RunScalars* run, hipStream_t s);

// t += dt; step += 1.
hipError_t launch_advance(RunScalars* run, hipStream_t s);

hipError_t launch_prim_to_state(const DeviceMesh& m, const float* prim, float* q, bool inverse,
                                hipStream_t s);

// Raise the dynamic-LDS limit of the stage kernels of order N (call once
// per process and device before any launch or capture).
hipError_t prepare_kernels(int N, int precision, int* blocks_per_cu);

// The contraction operator A = [-Dr -Ds -Dt | LIFT] of order N, transposed
// and padded in the layout the stage kernel reads (FP32).
std::vector<float> pack_operator(int N, const double* Dr, const double* Ds, const double* Dt,
                                 const double* LIFT);

// Split-BF16 volume operator -[Dr Ds Dt]: hi = bf16(x), lo = bf16(x - hi),
// laid out [hi|lo][MP][k-blocks of 32] as the split-BF16 stage kernel reads it.
std::vector<uint16_t> pack_operator_bf16(int N, const double* Dr, const double* Ds,
                                         const double* Dt);

// Bytes of dynamic LDS one stage block uses at order N (0 if unsupported).
size_t stage_lds_bytes(int N);

}  // namespace dg
