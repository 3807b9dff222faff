// Pressure probes and amplitude spectra (gfx950).
//
// Probe sampling: one wavefront per probe; lane i holds node i of the
// probe's element (Np <= 56 < 64), forms w_i q'_i for the five conserved
// perturbations, and the wavefront sums them with butterfly shuffles; lane 0
// turns the interpolated perturbation into p' with the perturbation-form
// pressure of Eq. 2 and stores it.
//
// Spectra: one thread per frequency bin k of one signal, a direct discrete
// Fourier sum over the samples with the phase index (k j mod n) carried as an
// integer (so the phase argument stays exact for any length), FP64 phases and
// accumulation; amplitude 2|X_k|/n (|X_k|/n at k = 0 and k = n/2), in dB.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "physics.hpp"
#include "probes.hpp"

namespace dg {
namespace {

__global__ __launch_bounds__(256) void probe_kernel(const ProbeSet* __restrict__ S, Phys P,
                                                    const float* __restrict__ q, float* out,
                                                    const RunScalars* run) {
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int n = S->n, Np = S->Np;
  if (p >= n) return;
  const int64_t k = S->elem[p];
  const float wi = lane < Np ? S->w[size_t(p) * Np + lane] : 0.0f;
  float acc[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    float x = lane < Np ? wi * q[(size_t(k) * 5 + v) * Np + lane] : 0.0f;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    acc[v] = x;
  }
  if (lane == 0) {
    Prim w;
    primitive<true>(P, acc, w);
    if (out) {
      out[p] = w.pp;
    } else {
      const int64_t j = run->step - 1;
      if (j >= 0 && j < S->cap) S->series[j * n + p] = w.pp;
    }
  }
}

__global__ __launch_bounds__(256) void spectrum_kernel(const float* __restrict__ x, int64_t n,
                                                       int32_t ns, double p_ref,
                                                       float* __restrict__ db) {
  const int s = blockIdx.y;
  const int64_t nk = n / 2 + 1;
  const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (k >= nk) return;
  double re = 0.0, im = 0.0;
  int64_t m = 0;  // k * j mod n
  const double two_over_n = 2.0 / double(n);
  for (int64_t j = 0; j < n; ++j) {
    // FP64 phase: an FP32 one is off by ~1e-7 rad, which is 0.01 dB on bins
    // 100 dB below the strongest
    double sn, cs;
    sincospi(two_over_n * double(m), &sn, &cs);
    const double xv = x[j * ns + s];
    re += xv * cs;
    im -= xv * sn;
    m += k;
    if (m >= n) m -= n;
  }
  const double scale = (k == 0 || 2 * k == n) ? 1.0 / double(n) : 2.0 / double(n);
  const double a = scale * sqrt(re * re + im * im);
  db[int64_t(s) * nk + k] = float(20.0 * log10(fmax(a, 1e-30 * p_ref) / p_ref));
}

}  // namespace

hipError_t launch_probe(const ProbeSet* dev_set, int n, const DeviceMesh& m, const float* q,
                        float* out, const RunScalars* run, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  probe_kernel<<<(n + 3) / 4, 256, 0, s>>>(dev_set, m.phys, q, out, run);
  return hipGetLastError();
}

hipError_t launch_spectrum(const float* x, int64_t n, int32_t n_signals, double p_ref, float* db,
                           hipStream_t s) {
  const int64_t nk = n / 2 + 1;
  dim3 grid(unsigned((nk + 255) / 256), unsigned(n_signals));
  spectrum_kernel<<<grid, 256, 0, s>>>(x, n, n_signals, p_ref, db);
  return hipGetLastError();
}

}  // namespace dg
