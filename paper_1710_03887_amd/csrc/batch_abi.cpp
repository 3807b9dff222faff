// C ABI of batched ensembles: several geometries x up to 16 members per
// persistent stage launch, one captured HIP graph per two steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/dg.h"
#include "batch.hpp"
#include "ctx.hpp"

namespace {

int bfail(dg_batch* b, int code, const std::string& m) {
  if (b) b->err = m;
  return code;
}

void bfree(dg_batch* b) {
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
  for (auto* p : b->scal) (void)hipFree(p);
  for (auto* p : b->partner) (void)hipFree(p);
  if (b->dev_geoms) (void)hipFree(b->dev_geoms);
  if (b->node_faces) (void)hipFree(b->node_faces);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
}

size_t state_floats(const dg_ctx* c) { return size_t(c->dm.K) * 5 * c->dm.Np * dg::kMembers; }

hipError_t enqueue_step(dg_batch* b, int parity0, hipStream_t s) {
  hipError_t e = dg::launch_batch_finalize(b->L, s);
  int parity = parity0;
  for (int i = 0; i < 5 && e == hipSuccess; ++i) {
    e = dg::launch_batch_stage(b->L, float(dg::kRK4a[i]), float(dg::kRK4b[i]), dg::kRK4c[i], parity, i == 4 ? 1 : 0, s);
    parity = 1 - parity;
  }
  if (e == hipSuccess) e = dg::launch_batch_advance(b->L, s);
  return e;
}

}  // namespace

extern "C" {

int dg_batch_create(dg_ctx* const* geoms, int ngeom, int members, void* stream, dg_batch** out) {
  if (!out) return DG_EINVAL;
  *out = nullptr;
  if (!geoms || ngeom < 1 || ngeom > 64 || members < 1 || members > dg::kMembers) return DG_EINVAL;
  for (int g = 0; g < ngeom; ++g)  // the batched kernel has no absorbing layer
    if (!geoms[g] || geoms[g]->host_only || geoms[g]->dm.sigma || geoms[g]->dm.scheme != 0 ||
        geoms[g]->curved.n != 0)
      return DG_EINVAL;
  const dg_ctx* c0 = geoms[0];
  for (int g = 1; g < ngeom; ++g) {
    const dg::Phys &a = c0->dm.phys, &p = geoms[g]->dm.phys;
    if (geoms[g]->dm.N != c0->dm.N || a.gamma != p.gamma || a.rho0 != p.rho0 || a.p0 != p.p0 ||
        a.u0[0] != p.u0[0] || a.u0[1] != p.u0[1] || a.u0[2] != p.u0[2] || a.alpha != p.alpha)
      return DG_EINVAL;
  }
  dg_batch* b = new (std::nothrow) dg_batch;
  if (!b) return DG_ENOMEM;
  b->geoms.assign(geoms, geoms + ngeom);
  b->members = members;
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto fail_out = [&](int code) {
    bfree(b);
    delete b;
    return code;
  };
  hipError_t e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return fail_out(DG_EHIP);

  // node -> faces bitmask
  const auto& ops = c0->ops;
  std::vector<uint8_t> nf(size_t(ops.Np), 0);
  for (int f = 0; f < 4; ++f)
    for (int i = 0; i < ops.Nfp; ++i) nf[size_t(ops.Fmask[size_t(f) * ops.Nfp + i])] |= uint8_t(1 << f);
  if (hipMalloc(&b->node_faces, nf.size()) != hipSuccess) return fail_out(DG_ENOMEM);
  if (hipMemcpyAsync(b->node_faces, nf.data(), nf.size(), hipMemcpyHostToDevice, s) != hipSuccess)
    return fail_out(DG_EHIP);

  int64_t first = 0;
  b->host_geoms.resize(ngeom);
  b->host_scal.resize(ngeom);
  for (int g = 0; g < ngeom; ++g) {
    const dg_ctx* c = geoms[g];
    dg::BatchGeom& G = b->host_geoms[g];
    std::memset(&G, 0, sizeof G);
    G.vgeo = c->dm.vgeo;
    G.sgeo = c->dm.sgeo;
    G.nbr = c->dm.nbr;
    G.finfo = c->dm.finfo;
    G.K = c->dm.K;
    G.first = first;
    first += c->dm.K;
    dg::BatchScalars* sc = nullptr;
    float* pb = nullptr;
    if (hipMalloc(&sc, sizeof(dg::BatchScalars)) != hipSuccess) return fail_out(DG_ENOMEM);
    b->scal.push_back(sc);
    if (hipMalloc(&pb, state_floats(c) * sizeof(float)) != hipSuccess) return fail_out(DG_ENOMEM);
    b->partner.push_back(pb);
    G.sc = sc;
    G.q[1] = pb;
  }
  if (hipMalloc(&b->dev_geoms, sizeof(dg::BatchGeom) * ngeom) != hipSuccess) return fail_out(DG_ENOMEM);

  dg::BatchLaunch& L = b->L;
  L.N = c0->dm.N;
  L.ngeom = ngeom;
  L.members = members;
  L.total = first;
  L.geoms = b->dev_geoms;
  L.Aop = c0->dm.Aop;
  L.fmask = c0->dm.fmask;
  L.nbr_node = c0->dm.nbr_node;
  L.node_faces = b->node_faces;
  L.phys = c0->dm.phys;
  L.num_cu = c0->dm.num_cu;
  L.waves_per_block = 4;
  if (dg::prepare_batch_kernels(L.N, 4, &L.blocks_per_cu) != hipSuccess) return fail_out(DG_EHIP);
  b->max_blocks_per_cu = L.blocks_per_cu;
  if (hipStreamSynchronize(s) != hipSuccess) return fail_out(DG_EHIP);
  *out = b;
  return DG_OK;
}

int dg_batch_destroy(dg_batch* b) {
  if (!b) return DG_OK;
  bfree(b);
  delete b;
  return DG_OK;
}

const char* dg_batch_last_error(const dg_batch* b) { return b ? b->err.c_str() : ""; }

int dg_batch_set_launch(dg_batch* b, int blocks_per_cu, int waves_per_block) {
  if (!b) return DG_EINVAL;
  if (blocks_per_cu < 0 || (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4 &&
                            waves_per_block != 8))
    return bfail(b, DG_EINVAL, "blocks_per_cu >= 0, waves_per_block in {1,2,4,8}");
  int maxb = 1;
  hipError_t e = dg::prepare_batch_kernels(b->L.N, waves_per_block, &maxb);
  if (e != hipSuccess) return bfail(b, DG_EHIP, hipGetErrorString(e));
  b->L.waves_per_block = waves_per_block;
  b->max_blocks_per_cu = maxb;
  b->L.blocks_per_cu = blocks_per_cu == 0 ? maxb : std::min(blocks_per_cu, maxb);
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
  return DG_OK;
}

int dg_batch_run(dg_batch* b, float* const* q, float* const* res, const double* amps, int64_t nsteps,
                 double cfl, double* t_inout, void* stream) {
  if (!b) return DG_EINVAL;
  if (!q || !res || !amps || !t_inout || nsteps < 0 || !(cfl > 0.0))
    return bfail(b, DG_EINVAL, "bad argument");
  const int ng = b->L.ngeom;
  hipStream_t s = static_cast<hipStream_t>(stream);
  bool same = b->graph != nullptr;
  for (int g = 0; g < ng; ++g) {
    if (!q[g] || !res[g]) return bfail(b, DG_EINVAL, "null state pointer");
    dg::BatchGeom& G = b->host_geoms[g];
    if (G.q[0] != q[g] || G.res != res[g]) same = false;
    G.q[0] = q[g];
    G.res = res[g];
    for (int m = 0; m < dg::kMembers; ++m) G.amp[m] = m < b->members ? float(amps[g * dg::kMembers + m]) : 0.0f;
    dg::BatchScalars& sc = b->host_scal[g];
    std::memset(&sc, 0, sizeof sc);
    sc.cfl = cfl;
    for (int m = 0; m < dg::kMembers; ++m) {
      sc.t[m] = t_inout[g * dg::kMembers + m];
      sc.first_bad[m] = -1;
    }
    hipError_t e = hipMemcpyAsync(b->scal[g], &sc, sizeof sc, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return bfail(b, DG_EHIP, hipGetErrorString(e));
  }
  hipError_t e = hipMemcpyAsync(b->dev_geoms, b->host_geoms.data(), sizeof(dg::BatchGeom) * ng,
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = dg::launch_batch_rate(b->L, 0, s);
  if (e != hipSuccess) return bfail(b, DG_EHIP, hipGetErrorString(e));

  if (nsteps >= 2 && !same) {
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bfail(b, DG_EHIP, hipGetErrorString(e));
    hipError_t le = enqueue_step(b, 0, b->capture_stream);
    if (le == hipSuccess) le = enqueue_step(b, 1, b->capture_stream);
    hipGraph_t gr = nullptr;
    e = hipStreamEndCapture(b->capture_stream, &gr);
    if (le != hipSuccess || e != hipSuccess) {
      if (gr) (void)hipGraphDestroy(gr);
      return bfail(b, DG_EHIP, hipGetErrorString(le != hipSuccess ? le : e));
    }
    e = hipGraphInstantiate(&b->graph, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) return bfail(b, DG_EHIP, hipGetErrorString(e));
  }
  for (int64_t k = 0; k + 1 < nsteps; k += 2) {
    e = hipGraphLaunch(b->graph, s);
    if (e != hipSuccess) return bfail(b, DG_EHIP, hipGetErrorString(e));
  }
  if (nsteps % 2 == 1) {
    e = enqueue_step(b, 0, s);
    for (int g = 0; g < ng && e == hipSuccess; ++g)
      e = hipMemcpyAsync(q[g], b->partner[g], state_floats(b->geoms[g]) * sizeof(float),
                         hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return bfail(b, DG_EHIP, hipGetErrorString(e));
  }
  for (int g = 0; g < ng && e == hipSuccess; ++g)
    e = hipMemcpyAsync(&b->host_scal[g], b->scal[g], sizeof(dg::BatchScalars), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return bfail(b, DG_EHIP, hipGetErrorString(e));
  b->first_bad.assign(size_t(ng) * dg::kMembers, -1);
  bool bad = false;
  for (int g = 0; g < ng; ++g)
    for (int m = 0; m < dg::kMembers; ++m) {
      t_inout[g * dg::kMembers + m] = b->host_scal[g].t[m];
      const int64_t fb = m < b->members ? b->host_scal[g].first_bad[m] : -1;
      b->first_bad[size_t(g) * dg::kMembers + m] = fb;
      if (fb >= 0) bad = true;
    }
  if (bad) return bfail(b, DG_ENONPHYS, "non-physical state in a member");
  return DG_OK;
}

int dg_batch_first_bad(const dg_batch* b, int64_t* steps) {
  if (!b || !steps) return DG_EINVAL;
  for (size_t i = 0; i < b->first_bad.size(); ++i) steps[i] = b->first_bad[i];
  return DG_OK;
}

}  // extern "C"
