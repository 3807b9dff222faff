// Host-side state of a context, shared by the single-solve and batched C ABI
// translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "batch.hpp"
#include "curved.hpp"
#include "kernels.hpp"
#include "mlp.hpp"
#include "probes.hpp"
#include "quad.hpp"
#include "setup.hpp"

namespace dg {

// Five-stage, fourth-order low-storage RK coefficients (Carpenter & Kennedy
// 1994), 2N-storage form: res = a_i res + dt L(q, t + c_i dt); q += b_i res.
constexpr double kRK4a[5] = {0.0, -567301805773.0 / 1357537059087.0,
                             -2404267990393.0 / 2016746695238.0,
                             -3550918686646.0 / 2091501179385.0,
                             -1275806237668.0 / 842570457699.0};
constexpr double kRK4b[5] = {1432997174477.0 / 9575080441755.0,
                             5161836677717.0 / 13612068292357.0,
                             1720146321549.0 / 2090206949498.0,
                             3134564353537.0 / 4481467310338.0,
                             2277821191437.0 / 14882151754819.0};
constexpr double kRK4c[5] = {0.0, 1432997174477.0 / 9575080441755.0,
                             2526269341429.0 / 6820363962896.0,
                             2006345519317.0 / 3224310063776.0,
                             2802321613138.0 / 2924317926251.0};

struct GraphCache {
  hipGraphExec_t exec = nullptr;
  const float* q = nullptr;
  const float* res = nullptr;
};

}  // namespace dg

struct dg_mlp;

struct dg_ctx {
  std::string err;
  dg_mlp* mlp = nullptr;            // attached learned closure, or null
  dg::LearnedBC lbc;                // its device tables (lface, ghost) and window
  std::vector<int32_t> lface_host;  // learned faces k * 4 + f, in nbr-index order
  int max_blocks_per_cu = 1;        // occupancy limit of the stage kernel
  bool host_only = false;
  dg::RefOps ops;
  dg::HostMesh mesh;
  dg::DeviceMesh dm;
  std::vector<void*> allocs;
  float* qbuf = nullptr;            // ping-pong partner of the caller's state
  dg::RunScalars* run = nullptr;    // device scalars
  dg::RunScalars host_run{};        // staging for uploads/downloads
  hipStream_t capture_stream = nullptr;
  dg::GraphCache two_steps;
  dg::GraphCache probe_steps;       // two steps with probe recording
  dg::ProbeSet probe_host{};        // staging of the device probe set
  dg::ProbeSet* probe_dev = nullptr;
  int64_t* probe_elem = nullptr;    // device [n]
  float* probe_w = nullptr;         // device [n][Np]
  int64_t last_bad = -1;
  dg::CurvedSet curved;             // curved elements (n = 0: none)
  std::vector<void*> curved_allocs;
  std::vector<int64_t> curved_elem_host;  // the curved elements, ascending
  std::vector<double> curved_x_host;      // their node positions [n][Np][3]
};

// Captured step graphs are rebuilt after anything they bake in changes
// (kernel variant, launch shape, learned closure, probes).
inline void drop_graphs(dg_ctx* c) {
  if (c->two_steps.exec) (void)hipGraphExecDestroy(c->two_steps.exec);
  c->two_steps = dg::GraphCache{};
  if (c->probe_steps.exec) (void)hipGraphExecDestroy(c->probe_steps.exec);
  c->probe_steps = dg::GraphCache{};
}

struct dg_batch {
  std::string err;
  std::vector<dg_ctx*> geoms;
  int members = dg::kMembers;
  dg::BatchLaunch L;
  std::vector<dg::BatchGeom> host_geoms;
  dg::BatchGeom* dev_geoms = nullptr;
  std::vector<dg::BatchScalars*> scal;     // device, one per geometry
  std::vector<float*> partner;             // ping-pong partners, one per geometry
  std::vector<dg::BatchScalars> host_scal;
  uint8_t* node_faces = nullptr;
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  int max_blocks_per_cu = 1;
  std::vector<int64_t> first_bad;
};

struct dg_mlp {
  std::string err;
  float* P = nullptr;        // parameters [kMlpParams]
  float* grads = nullptr;
  float* m = nullptr;        // Adam moments
  float* v = nullptr;
  uint16_t* Wb = nullptr;    // BF16 weights (padded layout)
  float* loss_dev = nullptr;
  int64_t t = 0;             // Adam steps taken
  bool bf16_stale = true;
  dg::MlpWork w;
};

namespace dg {
// Brings the BF16 weights of `m` up to date on stream s.
hipError_t mlp_sync_bf16(dg_mlp* m, hipStream_t s);
}  // namespace dg
