// C ABI of the nodal DG Euler library: context setup, uploads, launches and
// the HIP-graph-captured run loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/dg.h"
#include "ctx.hpp"

namespace {

thread_local std::string g_setup_error;

}  // namespace

namespace {

int fail(dg_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  else g_setup_error = msg;
  return code;
}

int hip_fail(dg_ctx* c, hipError_t e, const char* what) {
  return fail(c, DG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <class T>
int upload(dg_ctx* c, const T* host, size_t n, T** dev, hipStream_t s) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, n * sizeof(T) + 16);
  if (e != hipSuccess) return fail(c, DG_ENOMEM, "hipMalloc failed");
  c->allocs.push_back(p);
  if (host) {
    e = hipMemcpyAsync(p, host, n * sizeof(T), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync");
  }
  *dev = static_cast<T*>(p);
  return DG_OK;
}

void free_probes(dg_ctx* c) {
  if (c->probe_elem) (void)hipFree(c->probe_elem);
  if (c->probe_w) (void)hipFree(c->probe_w);
  if (c->probe_dev) (void)hipFree(c->probe_dev);
  c->probe_elem = nullptr;
  c->probe_w = nullptr;
  c->probe_dev = nullptr;
  c->probe_host = dg::ProbeSet{};
}

void free_curved(dg_ctx* c) {
  for (void* p : c->curved_allocs) (void)hipFree(p);
  c->curved_allocs.clear();
  c->curved = dg::CurvedSet{};
  c->dm.curved_flag = nullptr;
  c->curved_elem_host.clear();
  c->curved_x_host.clear();
}

void free_device(dg_ctx* c) {
  drop_graphs(c);
  free_probes(c);
  free_curved(c);
  for (void* p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  c->capture_stream = nullptr;
}

int need_device(dg_ctx* c) {
  if (!c) return fail(nullptr, DG_EINVAL, "null context");
  if (c->host_only) return fail(c, DG_ENODEV, "context was created host-only");
  return DG_OK;
}

int build_device(dg_ctx* c, hipStream_t s) {
  const auto& ops = c->ops;
  const auto& mh = c->mesh;
  const int Np = ops.Np, Nfp = ops.Nfp;
  const int64_t K = mh.K;
  const std::vector<float> Aop =
      dg::pack_operator(c->dm.N, ops.Dr.data(), ops.Ds.data(), ops.Dt.data(), ops.LIFT.data());
  std::vector<uint8_t> fmask(size_t(4) * Nfp);
  for (size_t i = 0; i < fmask.size(); ++i) fmask[i] = uint8_t(ops.Fmask[i]);
  std::vector<double> sgeo(size_t(K) * 16);
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 4; ++f) {
      for (int d = 0; d < 3; ++d) sgeo[size_t(k) * 16 + f * 4 + d] = mh.nrm[size_t(k) * 12 + f * 3 + d];
      sgeo[size_t(k) * 16 + f * 4 + 3] = mh.Fscale[size_t(k) * 4 + f];
    }
  // FP32 geometry of the tile-cooperative stage kernel: per tile of 16
  // elements, component-major [25][16], zero past the last element
  const int64_t ntiles = (K + 15) / 16;
  std::vector<float> geo32(size_t(ntiles) * 16 * 25, 0.0f);
  for (int64_t k = 0; k < K; ++k) {
    float* g = &geo32[size_t(k / 16) * 400 + size_t(k % 16)];
    for (int i = 0; i < 9; ++i) g[i * 16] = float(mh.drst_dx[size_t(k) * 9 + i]);
    for (int j = 0; j < 16; ++j) g[(9 + j) * 16] = float(sgeo[size_t(k) * 16 + j]);
  }
  std::vector<int32_t> nbr(size_t(K) * 4);
  std::vector<uint8_t> finfo(size_t(K) * 4);
  c->lface_host.clear();
  for (size_t i = 0; i < nbr.size(); ++i) {
    if (mh.EToE[i] >= 0) {
      nbr[i] = mh.EToE[i];
    } else if (mh.bc[i] == DG_BC_LEARNED) {   // -(tag + 8 * index of the learned face)
      nbr[i] = -int32_t(DG_BC_LEARNED + 8 * c->lface_host.size());
      c->lface_host.push_back(int32_t(i));
    } else {
      nbr[i] = -int32_t(mh.bc[i]);
    }
    finfo[i] = uint8_t(mh.EToF[i] | (mh.orient[i] << 2));
  }

  hipError_t e = dg::prepare_kernels(c->dm.N, c->dm.precision, &c->dm.blocks_per_cu);
  if (e != hipSuccess) return hip_fail(c, e, "stage kernel attributes");
  c->max_blocks_per_cu = c->dm.blocks_per_cu;
  int dev = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&c->dm.num_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(c, e, "device attributes");
  e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamCreate");

  float* dA;
  uint8_t *dF, *dNN, *dFi;
  double *dV, *dS;
  int32_t* dN;
  int rc;
  if ((rc = upload(c, Aop.data(), Aop.size(), &dA, s))) return rc;
  if (c->dm.precision == DG_SPLIT_BF16) {
    const std::vector<uint16_t> Abf =
        dg::pack_operator_bf16(c->dm.N, ops.Dr.data(), ops.Ds.data(), ops.Dt.data());
    uint16_t* dAb;
    if ((rc = upload(c, Abf.data(), Abf.size(), &dAb, s))) return rc;
    c->dm.Abf = dAb;
  }
  if ((rc = upload(c, fmask.data(), fmask.size(), &dF, s))) return rc;
  if ((rc = upload(c, ops.nbr_node.data(), ops.nbr_node.size(), &dNN, s))) return rc;
  if ((rc = upload(c, mh.drst_dx.data(), mh.drst_dx.size(), &dV, s))) return rc;
  if ((rc = upload(c, sgeo.data(), sgeo.size(), &dS, s))) return rc;
  float* dG32;
  if ((rc = upload(c, geo32.data(), geo32.size(), &dG32, s))) return rc;
  c->dm.geo32 = dG32;
  if ((rc = upload(c, nbr.data(), nbr.size(), &dN, s))) return rc;
  if ((rc = upload(c, finfo.data(), finfo.size(), &dFi, s))) return rc;
  if ((rc = upload<float>(c, nullptr, size_t(K) * 5 * Np, &c->qbuf, s))) return rc;
  if (int64_t(c->lface_host.size()) > INT32_MAX / (5LL * Np))
    return fail(c, DG_EINVAL, "learned faces x 5 x Np exceeds 2^31 - 1 (32-bit trace offsets)");
  if (!c->lface_host.empty()) {
    int32_t* dLf;
    float* dGh;
    const int64_t nl = int64_t(c->lface_host.size());
    if ((rc = upload(c, c->lface_host.data(), c->lface_host.size(), &dLf, s))) return rc;
    if ((rc = upload<float>(c, nullptr, size_t(nl) * 5 * Np, &dGh, s))) return rc;
    c->lbc.lface = dLf;
    c->lbc.ghost = dGh;
    c->lbc.nl = nl;
  }
  if (c->dm.scheme == 1) {
    dg::QuadOps Q;
    const std::string msg = dg::build_quadrature(ops, Q);
    if (!msg.empty()) return fail(c, DG_EINVAL, msg);
    std::vector<float> tab;
    for (const auto* v : {&Q.Bv, &Q.Dw, &Q.Bf, &Q.Lq, &Q.Bnb})
      for (double x : *v) tab.push_back(float(x));
    if (tab.size() != dg::quad_table_floats(c->dm.N)) return fail(c, DG_EINVAL, "quadrature table size");
    float* dT;
    if ((rc = upload(c, tab.data(), tab.size(), &dT, s))) return rc;
    c->dm.qtab = dT;
  }
  if ((rc = upload<dg::RunScalars>(c, nullptr, 1, &c->run, s))) return rc;
  c->host_run = dg::RunScalars{};
  c->host_run.first_bad = -1;
  e = hipMemcpyAsync(c->run, &c->host_run, sizeof(dg::RunScalars), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");

  c->dm.Aop = dA;
  c->dm.fmask = dF;
  c->dm.nbr_node = dNN;
  c->dm.vgeo = dV;
  c->dm.sgeo = dS;
  c->dm.nbr = dN;
  c->dm.finfo = dFi;
  return DG_OK;
}

// One stage launch, preceded by the learned ghost traces of q_in when a
// network is attached.
hipError_t stage(dg_ctx* c, int mode, const float* q_in, float* q_out, float* res, float* out,
                 float a, float b, double cc, double t, double dt, dg::RunScalars* run,
                 int rate_out, hipStream_t s) {
  if (c->mlp) {
    hipError_t e = dg::mlp_sync_bf16(c->mlp, s);
    if (e == hipSuccess) e = dg::launch_learned_ghost(c->dm, c->lbc, q_in, s);
    if (e != hipSuccess) return e;
  }
  if (c->curved.n == 0)
    return dg::launch_stage(c->dm, mode, q_in, q_out, res, out, a, b, cc, t, dt, run, rate_out, s);
  // curved elements: the stage kernel leaves their outputs and their share
  // of the time-step rate to their own pass
  hipError_t e = dg::launch_stage(c->dm, mode, q_in, q_out, res, out, a, b, cc, t, dt, run,
                                  rate_out, s);
  if (e == hipSuccess)
    e = dg::launch_curved(c->curved, c->dm, mode, q_in, q_out, res, out, a, b, cc, t, dt, run,
                          rate_out, s);
  return e;
}

// Enqueue one LSERK step on `s` with state ping-ponging between q and the
// context buffer; returns with the state in q when `end_in_q`, which needs
// an even number of stage swaps in total (handled by the caller).
hipError_t enqueue_stages(dg_ctx* c, float* q, float* res, bool start_in_q, double t, double dt,
                          dg::RunScalars* run, hipStream_t s) {
  float* bufs[2] = {q, c->qbuf};
  int cur = start_in_q ? 0 : 1;
  for (int i = 0; i < 5; ++i) {
    // the last stage of a run step also reduces the next step's CFL rate
    hipError_t e = stage(c, dg::MODE_STAGE, bufs[cur], bufs[1 - cur], res, nullptr,
                                    float(dg::kRK4a[i]), float(dg::kRK4b[i]), dg::kRK4c[i], t, dt, run,
                                    i == 4 ? 1 : 0, s);
    if (e != hipSuccess) return e;
    cur = 1 - cur;
  }
  return hipSuccess;
}

// One two-stage second-order Runge-Kutta step of the quadrature scheme
// (strong-stability-preserving form): q1 = q + dt L(q, t);
// q <- (q + q1 + dt L(q1, t + dt)) / 2.  The state ends in q.
hipError_t enqueue_rk2(dg_ctx* c, float* q, double t, double dt, dg::RunScalars* run,
                       hipStream_t s) {
  hipError_t e = dg::launch_quad(c->dm, dg::MODE_STAGE, q, nullptr, c->qbuf, nullptr, 0.0f, 1.0f,
                                 0.0, t, dt, run, 0, s);
  if (e == hipSuccess)
    e = dg::launch_quad(c->dm, dg::MODE_STAGE, c->qbuf, q, q, nullptr, 0.5f, 0.5f, 1.0, t, dt,
                        run, 1, s);
  return e;
}

}  // namespace

extern "C" {

int dg_mesh_setup(const dg_mesh_desc* d, void* stream, dg_ctx** out) {
  if (!out) return fail(nullptr, DG_EINVAL, "null output pointer");
  *out = nullptr;
  if (!d || !d->xyz || !d->EToV || !d->bc) return fail(nullptr, DG_EINVAL, "null mesh array");
  if (d->N < 1 || d->N > 5) return fail(nullptr, DG_EINVAL, "N must be in 1..5");
  if (d->K <= 0) return fail(nullptr, DG_EINVAL, "K must be positive");
  // the tile-cooperative stage kernel forms its exterior-trace offsets
  // (element x 5 Np + node) in 32 bits
  const int64_t state_len = 5LL * (d->N + 1) * (d->N + 2) * (d->N + 3) / 6;
  if (d->K > INT32_MAX / state_len)
    return fail(nullptr, DG_EINVAL, "K x 5 x Np exceeds 2^31 - 1 (32-bit state offsets)");
  if (d->precision != DG_FP32 && d->precision != DG_SPLIT_BF16)
    return fail(nullptr, DG_EINVAL, "unknown precision");
  if ((d->flags & ~(DG_SETUP_HOST_ONLY | DG_SETUP_QUADRATURE)) != 0)
    return fail(nullptr, DG_EINVAL, "unknown flags");
  const bool quad = (d->flags & DG_SETUP_QUADRATURE) != 0;
  if (quad && (d->N > 2 || d->precision != DG_FP32))
    return fail(nullptr, DG_EINVAL, "the quadrature scheme needs N <= 2 and the FP32 form");
  if (!(d->gamma > 1.0) || !(d->rho0 > 0.0) || !(d->p0 > 0.0))
    return fail(nullptr, DG_EINVAL, "need gamma > 1, rho0 > 0, p0 > 0");

  dg_ctx* c = new (std::nothrow) dg_ctx;
  if (!c) return fail(nullptr, DG_ENOMEM, "out of host memory");
  std::string msg = dg::build_reference(d->N, c->ops);
  if (msg.empty()) msg = dg::build_mesh(c->ops, d->K, d->xyz, d->EToV, d->bc, c->mesh);
  if (!msg.empty()) {
    delete c;
    const bool arg = msg.find("tag") != std::string::npos && msg.find("unknown") != std::string::npos;
    return fail(nullptr, arg ? DG_EINVAL : DG_EMESH, msg);
  }
  c->host_only = (d->flags & DG_SETUP_HOST_ONLY) != 0;
  c->dm.scheme = quad ? 1 : 0;
  c->dm.N = d->N;
  c->dm.Np = c->ops.Np;
  c->dm.Nfp = c->ops.Nfp;
  c->dm.K = d->K;
  c->dm.precision = d->precision;
  dg::Phys& P = c->dm.phys;
  P.gamma = float(d->gamma);
  P.gm1 = float(d->gamma - 1.0);
  P.rho0 = float(d->rho0);
  P.p0 = float(d->p0);
  const double c0 = std::sqrt(d->gamma * d->p0 / d->rho0);
  P.c0 = float(c0);
  P.Z0 = float(d->rho0 * c0);
  P.inv_c0sq = float(1.0 / (c0 * c0));
  double u2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    P.u0[k] = float(d->u0[k]);
    P.m0[k] = float(d->rho0 * d->u0[k]);
    u2 += d->u0[k] * d->u0[k];
  }
  P.E0 = float(d->p0 / (d->gamma - 1.0) + 0.5 * d->rho0 * u2);
  P.amp = float(d->inflow_amp);
  P.alpha = d->inflow_alpha > 0.0 ? d->inflow_alpha : 1.0;
  P.half_N1sq = float(0.5 * (d->N + 1) * (d->N + 1));
  if (!c->host_only) {
    const int rc = build_device(c, static_cast<hipStream_t>(stream));
    if (rc) {
      g_setup_error = c->err;
      free_device(c);
      delete c;
      return rc;
    }
  }
  *out = c;
  return DG_OK;
}

int dg_destroy(dg_ctx* c) {
  if (!c) return DG_OK;
  free_device(c);
  delete c;
  return DG_OK;
}

const char* dg_last_error(const dg_ctx* c) { return c ? c->err.c_str() : g_setup_error.c_str(); }

int dg_sizes(const dg_ctx* c, int32_t* Np, int32_t* Nfp, int64_t* K) {
  if (!c) return fail(nullptr, DG_EINVAL, "null context");
  if (Np) *Np = c->ops.Np;
  if (Nfp) *Nfp = c->ops.Nfp;
  if (K) *K = c->mesh.K;
  return DG_OK;
}

int dg_nodes(const dg_ctx* c, double* xyz_out) {
  if (!c || !xyz_out) return fail(const_cast<dg_ctx*>(c), DG_EINVAL, "null argument");
  dg::node_coordinates(c->ops, c->mesh, xyz_out);
  return DG_OK;
}

int dg_reference_operators(const dg_ctx* c, double* rst, double* Dr, double* Ds, double* Dt,
                           double* LIFT, int32_t* Fmask) {
  if (!c) return fail(nullptr, DG_EINVAL, "null context");
  const auto& o = c->ops;
  if (rst) std::memcpy(rst, o.rst.data(), o.rst.size() * sizeof(double));
  if (Dr) std::memcpy(Dr, o.Dr.data(), o.Dr.size() * sizeof(double));
  if (Ds) std::memcpy(Ds, o.Ds.data(), o.Ds.size() * sizeof(double));
  if (Dt) std::memcpy(Dt, o.Dt.data(), o.Dt.size() * sizeof(double));
  if (LIFT) std::memcpy(LIFT, o.LIFT.data(), o.LIFT.size() * sizeof(double));
  if (Fmask) std::memcpy(Fmask, o.Fmask.data(), o.Fmask.size() * sizeof(int32_t));
  return DG_OK;
}

int dg_geometry(const dg_ctx* c, double* drst_dx, double* J, double* nrm, double* Fscale,
                int64_t* mapP) {
  if (!c) return fail(nullptr, DG_EINVAL, "null context");
  const auto& m = c->mesh;
  if (drst_dx) std::memcpy(drst_dx, m.drst_dx.data(), m.drst_dx.size() * sizeof(double));
  if (J) std::memcpy(J, m.J.data(), m.J.size() * sizeof(double));
  if (nrm) std::memcpy(nrm, m.nrm.data(), m.nrm.size() * sizeof(double));
  if (Fscale) std::memcpy(Fscale, m.Fscale.data(), m.Fscale.size() * sizeof(double));
  if (mapP) dg::neighbour_map(c->ops, m, mapP);
  return DG_OK;
}

int dg_rhs(dg_ctx* c, const float* q, float* rhs, double t, void* stream) {
  int rc = need_device(c);
  if (rc) return rc;
  if (!q || !rhs) return fail(c, DG_EINVAL, "null state pointer");
  hipError_t e =
      c->dm.scheme == 1
          ? dg::launch_quad(c->dm, dg::MODE_RHS, q, nullptr, nullptr, rhs, 0.f, 0.f, 0.0, t, 0.0,
                            nullptr, 0, static_cast<hipStream_t>(stream))
          : stage(c, dg::MODE_RHS, q, nullptr, nullptr, rhs, 0.f, 0.f, 0.0, t, 0.0, nullptr, 0,
                  static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DG_OK : hip_fail(c, e, "stage launch");
}

int dg_step(dg_ctx* c, float* q, float* res, double t, double dt, void* stream) {
  int rc = need_device(c);
  if (rc) return rc;
  if (!q || !res) return fail(c, DG_EINVAL, "null state pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (c->dm.scheme == 1) {
    const hipError_t e = enqueue_rk2(c, q, t, dt, nullptr, s);
    return e == hipSuccess ? DG_OK : hip_fail(c, e, "stage launch");
  }
  hipError_t e = enqueue_stages(c, q, res, true, t, dt, nullptr, s);
  if (e != hipSuccess) return hip_fail(c, e, "stage launch");
  // five stages end in the context buffer
  e = hipMemcpyAsync(q, c->qbuf, size_t(c->dm.K) * 5 * c->dm.Np * sizeof(float),
                     hipMemcpyDeviceToDevice, s);
  return e == hipSuccess ? DG_OK : hip_fail(c, e, "hipMemcpyAsync");
}

int dg_stage(dg_ctx* c, const float* q_in, float* q_out, float* res, double a, double b,
             double t_stage, double dt, void* stream) {
  int rc = need_device(c);
  if (rc) return rc;
  if (!q_in || !q_out || !res) return fail(c, DG_EINVAL, "null state pointer");
  if (q_in == q_out) return fail(c, DG_EINVAL, "q_in and q_out must differ");
  if (c->dm.scheme == 1) return fail(c, DG_EINVAL, "no low-storage stage in the quadrature scheme");
  hipError_t e = stage(c, dg::MODE_STAGE, q_in, q_out, res, nullptr, float(a),
                                  float(b), 0.0, t_stage, dt, nullptr, 0,
                                  static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DG_OK : hip_fail(c, e, "stage launch");
}

int dg_stable_dt(dg_ctx* c, const float* q, double cfl, double* dt, void* stream) {
  int rc = need_device(c);
  if (rc) return rc;
  if (!q || !dt) return fail(c, DG_EINVAL, "null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  c->host_run = dg::RunScalars{};
  c->host_run.cfl = cfl;
  c->host_run.first_bad = -1;
  hipError_t e = hipMemcpyAsync(c->run, &c->host_run, sizeof(dg::RunScalars),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = dg::launch_rate(c->dm, q, c->run, s);
  if (e == hipSuccess) e = dg::launch_finalize(c->run, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&c->host_run, c->run, sizeof(dg::RunScalars), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "dg_stable_dt");
  *dt = c->host_run.dt;
  if (c->host_run.first_bad >= 0) return fail(c, DG_ENONPHYS, "non-physical state");
  return DG_OK;
}

namespace {

// The run loop; with `series`, the probe values of every step are recorded
// into series[step][probe] (probes set up, nsteps rows).
int run_impl(dg_ctx* c, float* q, float* res, int64_t nsteps, double cfl, double fixed_dt,
             double* t_inout, double* dt_last, hipStream_t s, float* series = nullptr) {
  c->host_run = dg::RunScalars{};
  c->host_run.t = *t_inout;
  c->host_run.cfl = cfl;
  c->host_run.fixed_dt = fixed_dt;
  c->host_run.first_bad = -1;
  if (c->mlp) {
    const hipError_t e = dg::mlp_sync_bf16(c->mlp, s);
    if (e != hipSuccess) return hip_fail(c, e, "learned closure weights");
  }
  hipError_t e = hipMemcpyAsync(c->run, &c->host_run, sizeof(dg::RunScalars),
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync");
  const int np = c->probe_host.n;
  if (series) {
    c->probe_host.series = series;
    c->probe_host.cap = nsteps;
    e = hipMemcpyAsync(c->probe_dev, &c->probe_host, sizeof(dg::ProbeSet), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync");
  }
  dg::GraphCache& gc = series ? c->probe_steps : c->two_steps;

  // the first step's CFL rate; every later one comes from the last stage
  // of the step before
  e = dg::launch_rate(c->dm, q, c->run, s);
  if (e != hipSuccess) return hip_fail(c, e, "rate launch");

  if (c->dm.scheme == 1) {  // quadrature scheme: a graph of one RK2 step, state stays in q
    if (nsteps >= 1 && (gc.q != q || !gc.exec)) {
      if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
      gc = dg::GraphCache{};
      hipStream_t cs = c->capture_stream;
      e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return hip_fail(c, e, "hipStreamBeginCapture");
      hipError_t le = dg::launch_finalize(c->run, cs);
      if (le == hipSuccess) le = enqueue_rk2(c, q, 0.0, 0.0, c->run, cs);
      if (le == hipSuccess) le = dg::launch_advance(c->run, cs);
      if (le == hipSuccess && series) le = dg::launch_probe(c->probe_dev, np, c->dm, q, nullptr, c->run, cs);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(cs, &g);
      if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(c, le, "launch during capture");
      }
      if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
      hipGraphExec_t ex = nullptr;
      e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
      gc.exec = ex;
      gc.q = q;
      gc.res = res;
    }
    for (int64_t k = 0; k < nsteps; ++k) {
      e = hipGraphLaunch(gc.exec, s);
      if (e != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
    }
    e = hipMemcpyAsync(&c->host_run, c->run, sizeof(dg::RunScalars), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(c, e, "dg_run sync");
    *t_inout = c->host_run.t;
    if (dt_last) *dt_last = c->host_run.dt;
    c->last_bad = c->host_run.first_bad;
    if (c->last_bad >= 0) return fail(c, DG_ENONPHYS, "non-physical state during dg_run");
    return DG_OK;
  }

  // a graph of two steps (ten stage swaps) leaves the state in q
  if (nsteps >= 2 && (gc.q != q || gc.res != res || !gc.exec)) {
    if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
    gc = dg::GraphCache{};
    hipStream_t cs = c->capture_stream;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamBeginCapture");
    hipError_t le = hipSuccess;
    for (int k = 0; k < 2 && le == hipSuccess; ++k) {
      le = dg::launch_finalize(c->run, cs);
      if (le == hipSuccess) le = enqueue_stages(c, q, res, k == 0, 0.0, 0.0, c->run, cs);
      if (le == hipSuccess) le = dg::launch_advance(c->run, cs);
      // the step's state is in the partner buffer after the first step, in q after the second
      if (le == hipSuccess && series)
        le = dg::launch_probe(c->probe_dev, np, c->dm, k == 0 ? c->qbuf : q, nullptr, c->run, cs);
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    if (le != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(c, le, "launch during capture");
    }
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
    gc.exec = ex;
    gc.q = q;
    gc.res = res;
  }
  for (int64_t k = 0; k + 1 < nsteps; k += 2) {
    e = hipGraphLaunch(gc.exec, s);
    if (e != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
  }
  if (nsteps % 2 == 1) {
    e = dg::launch_finalize(c->run, s);
    if (e == hipSuccess) e = enqueue_stages(c, q, res, true, 0.0, 0.0, c->run, s);
    if (e == hipSuccess) e = dg::launch_advance(c->run, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(q, c->qbuf, size_t(c->dm.K) * 5 * c->dm.Np * sizeof(float),
                         hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && series) e = dg::launch_probe(c->probe_dev, np, c->dm, q, nullptr, c->run, s);
    if (e != hipSuccess) return hip_fail(c, e, "single step");
  }
  e = hipMemcpyAsync(&c->host_run, c->run, sizeof(dg::RunScalars), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "dg_run sync");
  *t_inout = c->host_run.t;
  if (dt_last) *dt_last = c->host_run.dt;
  c->last_bad = c->host_run.first_bad;
  if (c->last_bad >= 0) return fail(c, DG_ENONPHYS, "non-physical state during dg_run");
  return DG_OK;
}

}  // namespace

int dg_run(dg_ctx* c, float* q, float* res, int64_t nsteps, double cfl, double* t_inout,
           double* dt_last, void* stream) {
  int rc = need_device(c);
  if (rc) return rc;
  if (!q || !res || !t_inout) return fail(c, DG_EINVAL, "null argument");
  if (nsteps < 0 || !(cfl > 0.0)) return fail(c, DG_EINVAL, "need nsteps >= 0 and cfl > 0");
  return run_impl(c, q, res, nsteps, cfl, 0.0, t_inout, dt_last, static_cast<hipStream_t>(stream));
}

int dg_run_fixed(dg_ctx* c, float* q, float* res, int64_t nsteps, double dt, double* t_inout,
                 void* stream) {
  int rc = need_device(c);
  if (rc) return rc;
  if (!q || !res || !t_inout) return fail(c, DG_EINVAL, "null argument");
  if (nsteps < 0 || !(dt > 0.0)) return fail(c, DG_EINVAL, "need nsteps >= 0 and dt > 0");
  return run_impl(c, q, res, nsteps, 1.0, dt, t_inout, nullptr, static_cast<hipStream_t>(stream));
}

int64_t dg_last_step(const dg_ctx* c) { return c ? c->last_bad : -1; }

int dg_set_kernel(dg_ctx* c, int variant) {
  int rc = need_device(c);
  if (rc) return rc;
  if (variant != 0 && variant != 1) return fail(c, DG_EINVAL, "variant must be 0 or 1");
  if (variant == 1 && (c->dm.scheme == 1 || !dg::spec_stage_supported(c->dm.N, c->dm.precision)))
    return fail(c, DG_EINVAL, "the role-specialized stage kernel needs the nodal scheme, the FP32 form and N <= 4");
  c->dm.variant = variant;
  drop_graphs(c);
  return DG_OK;
}

int dg_get_kernel(const dg_ctx* c) { return c ? c->dm.variant : -1; }

int dg_set_damping(dg_ctx* c, const float* sigma) {
  int rc = need_device(c);
  if (rc) return rc;
  if (c->dm.scheme == 1 && sigma) return fail(c, DG_EINVAL, "no absorbing layer in the quadrature scheme");
  c->dm.sigma = sigma;
  drop_graphs(c);
  return DG_OK;
}

int dg_set_curved(dg_ctx* c, const double* xyz_nodes, double tol, int64_t* n_curved_out,
                  void* stream) {
  if (!c) return fail(nullptr, DG_EINVAL, "null context");
  if (n_curved_out) *n_curved_out = 0;
  if (!c->host_only) drop_graphs(c);
  free_curved(c);
  if (!xyz_nodes) return DG_OK;
  if (!(tol > 0.0)) return fail(c, DG_EINVAL, "tol must be positive");
  if (c->dm.scheme == 1) return fail(c, DG_EINVAL, "no curved elements in the quadrature scheme");
  if (c->mlp) return fail(c, DG_EINVAL, "curved elements and a learned closure do not combine");
  std::vector<int64_t> elems;
  std::vector<float> vg, sg;
  const std::string msg = dg::curved_geometry(c->ops, c->mesh, xyz_nodes, tol, elems, vg, sg);
  if (!msg.empty()) return fail(c, DG_EINVAL, msg);
  const int64_t n = int64_t(elems.size());
  if (n == 0) return DG_OK;
  const int Np = c->ops.Np, NF = 4 * c->ops.Nfp;
  // host copies for locating probes in curved elements
  c->curved_elem_host = elems;
  c->curved_x_host.resize(size_t(n) * Np * 3);
  for (int64_t i = 0; i < n; ++i)
    std::copy(xyz_nodes + size_t(elems[i]) * Np * 3, xyz_nodes + size_t(elems[i] + 1) * Np * 3,
              c->curved_x_host.begin() + size_t(i) * Np * 3);
  if (c->host_only) {  // checked and kept for probe location only
    if (n_curved_out) *n_curved_out = n;
    return DG_OK;
  }
  // Dr, Ds, Dt each packed as the MFMA A operand (lane order, zero padded);
  // LIFT transposed, so that the lanes (one node each) read consecutive words
  const int MT = (Np + 15) / 16, KS = (Np + 3) / 4;
  std::vector<float> D(size_t(3) * KS * MT * 64, 0.0f), L(size_t(Np) * NF);
  const std::vector<double>* Da[3] = {&c->ops.Dr, &c->ops.Ds, &c->ops.Dt};
  for (int a = 0; a < 3; ++a)
    for (int ks = 0; ks < KS; ++ks)
      for (int t = 0; t < MT; ++t)
        for (int l = 0; l < 64; ++l) {
          const int row = 16 * t + (l & 15), j = 4 * ks + (l >> 4);
          if (row < Np && j < Np)
            D[((size_t(a) * KS + ks) * MT + t) * 64 + l] = float((*Da[a])[size_t(row) * Np + j]);
        }
  for (int n = 0; n < Np; ++n)
    for (int i = 0; i < NF; ++i) L[size_t(i) * Np + n] = float(c->ops.LIFT[size_t(n) * NF + i]);
  // per element: 1 for the curved ones (the stage kernels leave them alone)
  std::vector<uint8_t> flag(size_t(c->dm.K), 0);
  for (const int64_t k : elems) flag[size_t(k)] = 1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* p[6] = {};
  const size_t bytes[6] = {size_t(n) * sizeof(int64_t), vg.size() * sizeof(float),
                           sg.size() * sizeof(float), D.size() * sizeof(float),
                           L.size() * sizeof(float), flag.size()};
  const void* src[6] = {elems.data(), vg.data(), sg.data(), D.data(), L.data(), flag.data()};
  for (int i = 0; i < 6; ++i) {
    const hipError_t e = hipMalloc(&p[i], bytes[i]);
    if (e != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipFree(p[j]);
      free_curved(c);  // no half-set curved state (host copies included)
      return fail(c, DG_ENOMEM, "hipMalloc for curved elements");
    }
  }
  for (int i = 0; i < 6; ++i) c->curved_allocs.push_back(p[i]);
  hipError_t e = hipSuccess;
  for (int i = 0; i < 6 && e == hipSuccess; ++i)
    e = hipMemcpyAsync(p[i], src[i], bytes[i], hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host vectors end here
  if (e != hipSuccess) {
    free_curved(c);
    return hip_fail(c, e, "curved element upload");
  }
  c->curved.n = n;
  c->curved.elem = static_cast<const int64_t*>(p[0]);
  c->curved.vg = static_cast<const float*>(p[1]);
  c->curved.sg = static_cast<const float*>(p[2]);
  c->curved.D = static_cast<const float*>(p[3]);
  c->curved.L = static_cast<const float*>(p[4]);
  c->dm.curved_flag = static_cast<const uint8_t*>(p[5]);
  if (n_curved_out) *n_curved_out = n;
  return DG_OK;
}

int dg_probe_setup(dg_ctx* c, const double* xyz, int32_t n, int64_t* elements_out,
                   double* weights_out) {
  if (!c) return fail(nullptr, DG_EINVAL, "null context");
  if (!xyz || n < 1 || n > (1 << 20)) return fail(c, DG_EINVAL, "need 1 <= n <= 2^20 points");
  const int Np = c->ops.Np;
  std::vector<int64_t> elem(n);
  std::vector<float> w(size_t(n) * Np);
  std::vector<double> wd(Np);
  for (int32_t p = 0; p < n; ++p) {
    double rst[3];
    // with a curved set, a point whose straight-sided element is curved (or
    // that lies outside the straight-sided mesh) is located by inverting the
    // maps of the curved elements near it
    elem[p] = c->curved_elem_host.empty()
                  ? dg::locate_point(c->mesh, xyz + size_t(p) * 3, 1e-9, rst)
                  : dg::locate_point_curved(c->ops, c->mesh, c->curved_elem_host,
                                            c->curved_x_host.data(), xyz + size_t(p) * 3, 1e-9, rst);
    if (elem[p] == -2)
      return fail(c, DG_EINVAL, "probe " + std::to_string(p) + ": its curved element's map did not invert");
    if (elem[p] < 0) return fail(c, DG_EINVAL, "probe " + std::to_string(p) + " lies outside the mesh");
    dg::interpolation_weights(c->ops, rst, wd.data());
    for (int i = 0; i < Np; ++i) w[size_t(p) * Np + i] = float(wd[i]);
    if (weights_out) std::copy(wd.begin(), wd.end(), weights_out + size_t(p) * Np);
  }
  if (elements_out) std::copy(elem.begin(), elem.end(), elements_out);
  if (c->host_only) return DG_OK;  // located and weighed only
  drop_graphs(c);
  free_probes(c);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&c->probe_elem), sizeof(int64_t) * n);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&c->probe_w), sizeof(float) * w.size());
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&c->probe_dev), sizeof(dg::ProbeSet));
  if (e != hipSuccess) {
    free_probes(c);
    return fail(c, DG_ENOMEM, "hipMalloc failed");
  }
  c->probe_host.n = n;
  c->probe_host.Np = Np;
  c->probe_host.elem = c->probe_elem;
  c->probe_host.w = c->probe_w;
  e = hipMemcpy(c->probe_elem, elem.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->probe_w, w.data(), sizeof(float) * w.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(c->probe_dev, &c->probe_host, sizeof(dg::ProbeSet), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_probes(c);
    return hip_fail(c, e, "probe upload");
  }
  return DG_OK;
}

int dg_probe_sample(dg_ctx* c, const float* q, float* out, void* stream) {
  int rc = need_device(c);
  if (rc) return rc;
  if (!q || !out) return fail(c, DG_EINVAL, "null argument");
  if (c->probe_host.n < 1) return fail(c, DG_EINVAL, "no probes set up");
  const hipError_t e = dg::launch_probe(c->probe_dev, c->probe_host.n, c->dm, q, out, nullptr,
                                        static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DG_OK : hip_fail(c, e, "probe launch");
}

int dg_run_probes(dg_ctx* c, float* q, float* res, int64_t nsteps, double dt, double* t_inout,
                  float* series, void* stream) {
  int rc = need_device(c);
  if (rc) return rc;
  if (!q || !res || !t_inout || !series) return fail(c, DG_EINVAL, "null argument");
  if (nsteps < 0 || !(dt > 0.0)) return fail(c, DG_EINVAL, "need nsteps >= 0 and dt > 0");
  if (c->probe_host.n < 1) return fail(c, DG_EINVAL, "no probes set up");
  return run_impl(c, q, res, nsteps, 1.0, dt, t_inout, nullptr, static_cast<hipStream_t>(stream),
                  series);
}

int dg_spectrum(const float* series, int64_t n_samples, int32_t n_signals, double p_ref, float* db,
                void* stream) {
  if (!series || !db) return fail(nullptr, DG_EINVAL, "null argument");
  if (n_samples < 2 || n_signals < 1 || n_signals > 65535 || !(p_ref > 0.0))
    return fail(nullptr, DG_EINVAL, "need n_samples >= 2, 1 <= n_signals <= 65535, p_ref > 0");
  const hipError_t e = dg::launch_spectrum(series, n_samples, n_signals, p_ref, db,
                                           static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DG_OK : hip_fail(nullptr, e, "spectrum launch");
}

int dg_set_launch(dg_ctx* c, int blocks_per_cu) {
  int rc = need_device(c);
  if (rc) return rc;
  if (blocks_per_cu < 0) return fail(c, DG_EINVAL, "blocks_per_cu must be >= 0");
  c->dm.blocks_per_cu = blocks_per_cu == 0 ? c->max_blocks_per_cu
                                           : std::min(blocks_per_cu, c->max_blocks_per_cu);
  drop_graphs(c);
  return DG_OK;
}

int dg_prim_to_state(dg_ctx* c, const float* prim, float* q, void* stream) {
  int rc = need_device(c);
  if (rc) return rc;
  if (!prim || !q) return fail(c, DG_EINVAL, "null argument");
  hipError_t e = dg::launch_prim_to_state(c->dm, prim, q, false, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DG_OK : hip_fail(c, e, "prim_to_state");
}

int dg_state_to_prim(dg_ctx* c, const float* q, float* prim, void* stream) {
  int rc = need_device(c);
  if (rc) return rc;
  if (!prim || !q) return fail(c, DG_EINVAL, "null argument");
  hipError_t e = dg::launch_prim_to_state(c->dm, q, prim, true, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DG_OK : hip_fail(c, e, "state_to_prim");
}

}  // extern "C"
