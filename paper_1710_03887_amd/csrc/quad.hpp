// The paper's discretization (Appendix A): the weak form with Gauss
// quadrature, advanced by a two-stage second-order Runge-Kutta scheme.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "kernels.hpp"

namespace dg {

// Floats of the packed FP32 tables of order N (Bv, Dw, Bf, Lq, Bnb in the
// QuadOps layouts, one after the other).
size_t quad_table_floats(int N);

// One right-hand side (mode MODE_RHS: out = L(q_in)) or one Runge-Kutta
// stage  q_out = alpha q_base + beta (q_in + dt L(q_in))  at the stage time
// t + c dt (run scalars when `run` is given, else t_host/dt_host); with
// rate_out the stage also reduces the next step's CFL rate from q_out.
// q_base may equal q_out (each element reads only its own q_base values).
hipError_t launch_quad(const DeviceMesh& m, int mode, const float* q_in, const float* q_base,
                       float* q_out, float* out, float alpha, float beta, double c,
                       double t_host, double dt_host, RunScalars* run, int rate_out,
                       hipStream_t s);

}  // namespace dg
