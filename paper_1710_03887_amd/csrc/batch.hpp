// Batched ensembles: several geometries x up to 16 members (pulse
// amplitudes) advanced together, member-innermost state layout.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace dg {

constexpr int kMembers = 16;  // members per geometry (MFMA n = 16)

// Per-geometry run scalars, one slot per member.
struct BatchScalars {
  double t[kMembers];
  double dt[kMembers];
  double cfl;
  int64_t step;
  int64_t first_bad[kMembers];
  uint32_t rate_bits[kMembers];
  uint32_t bad[kMembers];
};

// One geometry of a batch, as the batched stage kernel reads it.
struct BatchGeom {
  const double* vgeo;       // [K][9]
  const double* sgeo;       // [K][4][4]
  const int32_t* nbr;       // [K][4]
  const uint8_t* finfo;     // [K][4]
  int64_t K;
  int64_t first;            // first work item (element) of this geometry
  float* q[2];              // ping-pong states [K][5][Np][16]
  float* res;               // [K][5][Np][16]
  BatchScalars* sc;         // device scalars
  float amp[kMembers];      // inflow amplitude per member
};

struct BatchLaunch {
  int N = 0;
  int ngeom = 0;
  int members = kMembers;   // active members (columns >= members are zero)
  int64_t total = 0;        // total elements over all geometries
  const BatchGeom* geoms = nullptr;   // device array [ngeom]
  const float* Aop = nullptr;         // operator, pack_operator layout
  const uint8_t* fmask = nullptr;
  const uint8_t* nbr_node = nullptr;
  const uint8_t* node_faces = nullptr;  // [Np] bit f set when node is on face f
  Phys phys;                           // amp unused (per member)
  int num_cu = 256;
  int blocks_per_cu = 2;
  int waves_per_block = 4;
};

// One fused LSERK stage for every geometry and member.  parity selects
// q[parity] -> q[1 - parity]; rate_out makes the stage reduce each member's
// next CFL rate.  t/dt are read per member from each geometry's scalars.
hipError_t launch_batch_stage(const BatchLaunch& L, float a, float b, double c, int parity,
                              int rate_out, hipStream_t s);

// Per-member CFL rate of q[parity] (start of a run).
hipError_t launch_batch_rate(const BatchLaunch& L, int parity, hipStream_t s);

// dt = cfl / rate per member (or a fixed dt when fixed_dt > 0); t += dt.
hipError_t launch_batch_finalize(const BatchLaunch& L, hipStream_t s);
hipError_t launch_batch_advance(const BatchLaunch& L, hipStream_t s);

hipError_t prepare_batch_kernels(int N, int waves_per_block, int* blocks_per_cu);

}  // namespace dg
