// Pressure probes and amplitude spectra (Section 3: the pressure sampled at
// sensor points and its frequency content).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace dg {

// Device-resident probe set: probe p lies in element elem[p] and the
// solution there is sum_i w[p][i] q[elem[p]][v][i].  Recording runs write
// series[(step - 1) * n + p] after each step while step <= cap.
struct ProbeSet {
  int32_t n = 0;
  int32_t Np = 0;
  int64_t cap = 0;
  float* series = nullptr;       // [cap][n]
  const int64_t* elem = nullptr; // [n]
  const float* w = nullptr;      // [n][Np]
};

// p - p0 at each of the n probes: into out[p] when out is not null, else
// into the recording series at the run's step counter.
hipError_t launch_probe(const ProbeSet* dev_set, int n, const DeviceMesh& m, const float* q,
                        float* out, const RunScalars* run, hipStream_t s);

// One-sided amplitude spectra of n_signals real series x[j][s] (sample j,
// signal s), in dB relative to p_ref: db[s][k], k = 0 .. n/2.
hipError_t launch_spectrum(const float* x, int64_t n, int32_t n_signals, double p_ref, float* db,
                           hipStream_t s);

}  // namespace dg
