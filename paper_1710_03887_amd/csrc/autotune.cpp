// Launch-shape autotuner for the stage kernels.  Every candidate shape is
// timed with HIP events on the caller's stream over a few stage launches;
// the fastest is kept and recorded in a plain-text cache (one line per
// workload: key, two launch parameters, microseconds -- blocks per CU and
// stage-kernel variant for a single solution, blocks per CU and waves per
// block for an ensemble), so that a later process with the same workload and
// device skips the search.
// Results never depend on the launch shape: elements are independent and
// every reduction is a maximum.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/dg.h"
#include "ctx.hpp"

namespace {

constexpr int kWarm = 2, kReps = 8;

std::string device_key() {
  int dev = 0;
  hipDeviceProp_t p{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess)
    return "unknown";
  std::string arch = p.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch.resize(colon);
  return arch + "/cu" + std::to_string(p.multiProcessorCount);
}

bool cache_lookup(const char* path, const std::string& key, int* bpc, int* waves) {
  if (!path || !*path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    char* tab = std::strchr(line, '\t');
    if (!tab) continue;
    *tab = '\0';
    int a = 0, b = 0;
    double us = 0.0;
    if (key == line && std::sscanf(tab + 1, "%d\t%d\t%lf", &a, &b, &us) == 3) {
      *bpc = a;
      *waves = b;
      found = true;          // the last matching line wins
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const char* path, const std::string& key, int bpc, int waves, double us) {
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s\t%d\t%d\t%.3f\n", key.c_str(), bpc, waves, us);
  std::fclose(f);
}

// average microseconds per launch of `launch`, or a negative value on error
template <class F>
double time_launch(F&& launch, hipStream_t s, hipError_t* err) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double us = -1.0;
  *err = hipEventCreate(&e0);
  if (*err == hipSuccess) *err = hipEventCreate(&e1);
  for (int i = 0; i < kWarm && *err == hipSuccess; ++i) *err = launch();
  if (*err == hipSuccess) *err = hipEventRecord(e0, s);
  for (int i = 0; i < kReps && *err == hipSuccess; ++i) *err = launch();
  if (*err == hipSuccess) *err = hipEventRecord(e1, s);
  if (*err == hipSuccess) *err = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (*err == hipSuccess) *err = hipEventElapsedTime(&ms, e0, e1);
  if (*err == hipSuccess) us = 1e3 * double(ms) / kReps;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return us;
}

}  // namespace

extern "C" {

int dg_autotune(dg_ctx* c, const float* q, float* res, const char* cache_path, int* blocks_per_cu,
                void* stream) {
  if (!c) return DG_EINVAL;
  if (c->host_only) {
    c->err = "context was created host-only";
    return DG_ENODEV;
  }
  if (!q || !res) {
    c->err = "null state pointer";
    return DG_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (c->dm.scheme == 1) {  // the quadrature kernel has one launch shape
    if (blocks_per_cu) *blocks_per_cu = 0;
    return DG_OK;
  }
  const std::string key = "single/N" + std::to_string(c->dm.N) + "/K" + std::to_string(c->dm.K) +
                          "/prec" + std::to_string(c->dm.precision) + "/" + device_key();
  const bool wave_ok = dg::spec_stage_supported(c->dm.N, c->dm.precision);
  int best = 0, best_v = 0;
  if (!cache_lookup(cache_path, key, &best, &best_v) || best < 1 ||
      best > c->max_blocks_per_cu || best_v < 0 || best_v > 1 || (best_v == 1 && !wave_ok)) {
    double best_us = 1e300;
    // the tile-cooperative kernel at every residency, then the
    // role-specialized kernel (one block of eight wavefronts per CU)
    const int ncand = c->max_blocks_per_cu + (wave_ok ? 1 : 0);
    for (int cand = 0; cand < ncand; ++cand) {
      const int variant = cand < c->max_blocks_per_cu ? 0 : 1;
      const int bpc = variant == 0 ? cand + 1 : 1;
      c->dm.blocks_per_cu = bpc;
      c->dm.variant = variant;
      hipError_t err = hipSuccess;
      const double us = time_launch(
          [&] {
            // b = 0 leaves the state unchanged; res is overwritten
            return dg::launch_stage(c->dm, dg::MODE_STAGE, q, c->qbuf, res, nullptr,
                                    float(dg::kRK4a[1]), 0.0f, 0.0, 0.0, 0.0, nullptr, 0, s);
          },
          s, &err);
      if (err != hipSuccess) {
        c->err = std::string("autotune: ") + hipGetErrorString(err);
        return DG_EHIP;
      }
      if (us < best_us) {
        best_us = us;
        best = bpc;
        best_v = variant;
      }
    }
    cache_store(cache_path, key, best, best_v, best_us);
  }
  c->dm.blocks_per_cu = best;
  c->dm.variant = best_v;
  drop_graphs(c);
  if (blocks_per_cu) *blocks_per_cu = best;
  return DG_OK;
}

int dg_batch_autotune(dg_batch* b, float* const* q, float* const* res, const char* cache_path,
                      int* blocks_per_cu, int* waves_per_block, void* stream) {
  if (!b) return DG_EINVAL;
  const int ng = b->L.ngeom;
  if (!q || !res) {
    b->err = "null state pointer";
    return DG_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::string key = "batch/N" + std::to_string(b->L.N) + "/m" + std::to_string(b->members) + "/K";
  for (int g = 0; g < ng; ++g) key += (g ? "," : "") + std::to_string(b->host_geoms[g].K);
  key += "/" + device_key();

  int best_b = 0, best_w = 0;
  const bool cached = cache_lookup(cache_path, key, &best_b, &best_w);
  hipError_t err = hipSuccess;
  if (!cached || dg_batch_set_launch(b, best_b, best_w) != DG_OK) {
    // stage inputs: the caller's states, zero time step (the state is kept)
    for (int g = 0; g < ng; ++g) {
      if (!q[g] || !res[g]) {
        b->err = "null state pointer";
        return DG_EINVAL;
      }
      b->host_geoms[g].q[0] = q[g];
      b->host_geoms[g].res = res[g];
      std::memset(&b->host_scal[g], 0, sizeof(dg::BatchScalars));
      if (err == hipSuccess)
        err = hipMemcpyAsync(b->scal[g], &b->host_scal[g], sizeof(dg::BatchScalars),
                             hipMemcpyHostToDevice, s);
    }
    if (err == hipSuccess)
      err = hipMemcpyAsync(b->dev_geoms, b->host_geoms.data(), sizeof(dg::BatchGeom) * ng,
                           hipMemcpyHostToDevice, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    double best_us = 1e300;
    const int waves[4] = {1, 2, 4, 8};
    for (int wi = 0; wi < 4 && err == hipSuccess; ++wi) {
      int maxb = 1;
      err = dg::prepare_batch_kernels(b->L.N, waves[wi], &maxb);
      for (int bpc = 1; bpc <= maxb && err == hipSuccess; ++bpc) {
        b->L.waves_per_block = waves[wi];
        b->L.blocks_per_cu = bpc;
        const double us = time_launch(
            [&] {
              return dg::launch_batch_stage(b->L, float(dg::kRK4a[1]), 0.0f, 0.0, 0, 0, s);
            },
            s, &err);
        if (err == hipSuccess && us < best_us) {
          best_us = us;
          best_b = bpc;
          best_w = waves[wi];
        }
      }
    }
    if (err != hipSuccess) {
      b->err = std::string("autotune: ") + hipGetErrorString(err);
      return DG_EHIP;
    }
    cache_store(cache_path, key, best_b, best_w, best_us);
    const int rc = dg_batch_set_launch(b, best_b, best_w);
    if (rc != DG_OK) return rc;
  }
  if (blocks_per_cu) *blocks_per_cu = b->L.blocks_per_cu;
  if (waves_per_block) *waves_per_block = b->L.waves_per_block;
  return DG_OK;
}

}  // extern "C"
