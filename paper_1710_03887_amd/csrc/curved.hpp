// Curved (isoparametric) elements (Section 3: curved boundary faces in place
// of flat ones): per-node metric terms and per-face-node normals for the
// elements whose map is not affine, and the pass that evaluates their
// right-hand side after the stage kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace dg {

struct CurvedSet {
  int64_t n = 0;                 // curved elements
  const int64_t* elem = nullptr; // [n] element ids, ascending
  const float* vg = nullptr;     // [n][Np][9] d r_a / d x_d at each node
  const float* sg = nullptr;     // [n][4][Nfp][4] unit normal, sJ/J at each face node
  // Dr, Ds, Dt as the A operand of MFMA f32 16x16x4: [3][KS][MT][64], lane l
  // of (a, ks, t) = D_a[n][j] for row n = 16 t + l%16 and j = 4 ks + l/16
  // (zero outside Np rows and columns); MT = ceil(Np / 16), KS = ceil(Np / 4)
  const float* D = nullptr;
  const float* L = nullptr;      // [4 Nfp (i)][Np (n)] = LIFT[n][i] (transposed)
};

// The curved elements' share of one right-hand side or LSERK stage, with the
// contract of launch_stage (MODE_RHS: out = f(q_in); MODE_STAGE:
// res = a res + dt f(q_in), q_out = q_in + b res), after a stage kernel that
// left these elements' outputs alone (DeviceMesh::curved_flag); with run and
// rate_out set, also their share of the next step's time-step rate.
hipError_t launch_curved(const CurvedSet& cv, const DeviceMesh& m, int mode, const float* q_in,
                         float* q_out, float* res, float* out, float a, float b, double c,
                         double t_host, double dt_host, RunScalars* run, int rate_out,
                         hipStream_t s);

}  // namespace dg
