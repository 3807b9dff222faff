// C ABI of the learned boundary closure: network objects, FP32 training,
// BF16 inference, attaching a network to a context, trace sampling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <string>

#include "../../include/dg.h"
#include "ctx.hpp"
#include "mlp.hpp"

namespace {

constexpr float kBeta1 = 0.9f, kBeta2 = 0.999f, kAdamEps = 1e-8f, kLossEps = 1e-6f;

int mfail(dg_mlp* m, int code, const std::string& msg) {
  if (m) m->err = msg;
  return code;
}

void free_work(dg::MlpWork& w) {
  float* bufs[] = {w.x, w.y, w.z1, w.a1, w.z2, w.a2, w.yh, w.d3, w.d2, w.d1, w.lrow, w.lsum, w.part};
  for (float* b : bufs)
    if (b) (void)hipFree(b);
  w = dg::MlpWork{};
}

// workspace for at least B rows (allocates outside any capture)
hipError_t ensure_cap(dg_mlp* m, int64_t B) {
  if (B <= m->w.cap) return hipSuccess;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return e;
  free_work(m->w);
  const int64_t cap = std::max<int64_t>(B, 1024);
  dg::MlpWork& w = m->w;
  struct {
    float** p;
    int64_t n;
  } want[] = {{&w.x, cap * dg::kMlpIn},   {&w.y, cap * dg::kMlpOut}, {&w.z1, cap * dg::kMlpH},
              {&w.a1, cap * dg::kMlpH},   {&w.z2, cap * dg::kMlpH},  {&w.a2, cap * dg::kMlpH},
              {&w.yh, cap * dg::kMlpOut}, {&w.d3, cap * dg::kMlpOut}, {&w.d2, cap * dg::kMlpH},
              {&w.d1, cap * dg::kMlpH},   {&w.lrow, cap},             {&w.lsum, 1},
              {&w.part, dg::kMlpPartFloats}};
  for (auto& x : want) {
    e = hipMalloc(reinterpret_cast<void**>(x.p), size_t(x.n) * sizeof(float));
    if (e != hipSuccess) {
      free_work(w);
      return e;
    }
  }
  w.cap = cap;
  return hipSuccess;
}

void free_mlp(dg_mlp* m) {
  free_work(m->w);
  void* bufs[] = {m->P, m->grads, m->m, m->v, m->Wb, m->loss_dev};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
}

int read_loss(dg_mlp* m, float* loss, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(loss, m->loss_dev, sizeof(float), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? DG_OK : mfail(m, DG_EHIP, hipGetErrorString(e));
}

// Fixed activation storage of dg_mlp_infer_noalloc: z1, a1, z2, a2 of up to
// DG_MLP_NOALLOC_ROWS rows.  In host code `scratch` only names the symbol;
// its device address comes from hipGetSymbolAddress, once per device.
constexpr int64_t kNoAllocRows = DG_MLP_NOALLOC_ROWS;
constexpr size_t kScratchFloats = size_t(kNoAllocRows) * 4 * dg::kMlpH;
static __device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
float* scratch_dev[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.
hipError_t scratch_address(float** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_dev[dev] = static_cast<float*>(p);
  }
  *out = scratch_dev[dev];
  return hipSuccess;
}

}  // namespace

namespace dg {

hipError_t mlp_sync_bf16(dg_mlp* m, hipStream_t s) {
  if (!m->bf16_stale) return hipSuccess;
  const hipError_t e = mlp_pack_bf16(m->P, m->Wb, s);
  if (e == hipSuccess) m->bf16_stale = false;
  return e;
}

}  // namespace dg

extern "C" {

int dg_mlp_create(const float* params, void* stream, dg_mlp** out) {
  if (!out) return DG_EINVAL;
  *out = nullptr;
  if (!params) return DG_EINVAL;
  dg_mlp* m = new (std::nothrow) dg_mlp;
  if (!m) return DG_ENOMEM;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t bytes = size_t(dg::kMlpParams) * sizeof(float);
  hipError_t e = hipSuccess;
  void** bufs[] = {reinterpret_cast<void**>(&m->P), reinterpret_cast<void**>(&m->grads),
                   reinterpret_cast<void**>(&m->m), reinterpret_cast<void**>(&m->v)};
  for (void** b : bufs)
    if (e == hipSuccess) e = hipMalloc(b, bytes);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&m->Wb), size_t(dg::kBfTotal) * 2);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&m->loss_dev), sizeof(float));
  if (e == hipSuccess) e = hipMemcpyAsync(m->P, params, bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(m->m, 0, bytes, s);
  if (e == hipSuccess) e = hipMemsetAsync(m->v, 0, bytes, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    free_mlp(m);
    delete m;
    return e == hipErrorOutOfMemory ? DG_ENOMEM : DG_EHIP;
  }
  *out = m;
  return DG_OK;
}

int dg_mlp_destroy(dg_mlp* m) {
  if (!m) return DG_OK;
  (void)hipDeviceSynchronize();
  free_mlp(m);
  delete m;
  return DG_OK;
}

const char* dg_mlp_last_error(const dg_mlp* m) { return m ? m->err.c_str() : ""; }

int dg_mlp_get_params(dg_mlp* m, float* params, void* stream) {
  if (!m || !params) return DG_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(params, m->P, size_t(dg::kMlpParams) * sizeof(float),
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? DG_OK : mfail(m, DG_EHIP, hipGetErrorString(e));
}

int dg_mlp_set_params(dg_mlp* m, const float* params, void* stream) {
  if (!m || !params) return DG_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(m->P, params, size_t(dg::kMlpParams) * sizeof(float),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  m->bf16_stale = true;
  return e == hipSuccess ? DG_OK : mfail(m, DG_EHIP, hipGetErrorString(e));
}

int dg_mlp_infer(dg_mlp* m, const float* X, float* Y, int64_t B, int bf16, void* stream) {
  if (!m) return DG_EINVAL;
  if (!X || !Y || B < 0) return mfail(m, DG_EINVAL, "null pointer or negative row count");
  if (B == 0) return DG_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (bf16) {
    e = dg::mlp_sync_bf16(m, s);
    if (e == hipSuccess) e = dg::mlp_infer_bf16(m->Wb, m->P, X, B, Y, s);
  } else {
    e = ensure_cap(m, B);
    if (e == hipSuccess) e = dg::mlp_forward_f32(m->P, X, B, m->w, Y, s);
  }
  return e == hipSuccess ? DG_OK : mfail(m, DG_EHIP, hipGetErrorString(e));
}

int dg_mlp_infer_noalloc(dg_mlp* m, const float* X, float* Y, int64_t B, void* stream) {
  if (!m) return DG_EINVAL;
  if (B == 0) return DG_OK;  // nothing to do; X and Y are not read
  if (!X || !Y || B < 0) return mfail(m, DG_EINVAL, "null pointer or negative row count");
  if (B > kNoAllocRows)
    return mfail(m, DG_EINVAL, "dg_mlp_infer_noalloc: B = " + std::to_string(B) +
                                   " exceeds DG_MLP_NOALLOC_ROWS = " + std::to_string(kNoAllocRows));
  float* base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess)
    return mfail(m, DG_EHIP, std::string("scratch address: ") + hipGetErrorString(e));
  // the same four activation arrays as the allocated workspace, packed at B rows
  dg::MlpWork w;
  w.cap = B;
  w.z1 = base;
  w.a1 = base + B * dg::kMlpH;
  w.z2 = base + 2 * B * dg::kMlpH;
  w.a2 = base + 3 * B * dg::kMlpH;
  e = dg::mlp_forward_f32(m->P, X, B, w, Y, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DG_OK : mfail(m, DG_EHIP, hipGetErrorString(e));
}

int dg_mlp_grad(dg_mlp* m, const float* X, const float* Y, int64_t B, float* loss, float* grads,
                void* stream) {
  if (!m) return DG_EINVAL;
  if (!X || !Y || B <= 0) return mfail(m, DG_EINVAL, "null pointer or empty batch");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = ensure_cap(m, B);
  if (e == hipSuccess)
    e = dg::mlp_grad_f32(m->P, X, Y, B, kLossEps, m->w, grads ? grads : m->grads, m->loss_dev, s);
  if (e != hipSuccess) return mfail(m, DG_EHIP, hipGetErrorString(e));
  return loss ? read_loss(m, loss, s) : DG_OK;
}

int dg_mlp_train_step(dg_mlp* m, const float* X, const float* Y, int64_t n_rows,
                      const int64_t* rows, int64_t B, float lr, float* loss, void* stream) {
  if (!m) return DG_EINVAL;
  if (!X || !Y || B <= 0 || n_rows <= 0 || !(lr >= 0.0f) || (!rows && B > n_rows))
    return mfail(m, DG_EINVAL, "bad argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = ensure_cap(m, B);
  const float* x = X;
  const float* y = Y;
  if (e == hipSuccess && rows) {
    e = dg::mlp_gather_rows(X, Y, rows, B, n_rows, m->w, s);
    x = m->w.x;
    y = m->w.y;
  }
  if (e == hipSuccess) e = dg::mlp_grad_f32(m->P, x, y, B, kLossEps, m->w, m->grads, m->loss_dev, s);
  if (e == hipSuccess) {
    m->t += 1;
    const float c1 = float(1.0 / (1.0 - std::pow(double(kBeta1), double(m->t))));
    const float c2 = float(1.0 / (1.0 - std::pow(double(kBeta2), double(m->t))));
    e = dg::mlp_adam(m->P, m->grads, m->m, m->v, lr, kBeta1, kBeta2, kAdamEps, c1, c2, s);
    m->bf16_stale = true;
  }
  if (e != hipSuccess) return mfail(m, DG_EHIP, hipGetErrorString(e));
  return loss ? read_loss(m, loss, s) : DG_OK;
}

int dg_set_learned_bc(dg_ctx* c, dg_mlp* m, double norm, double p_lo, double p_hi,
                      double blend) {
  if (!c) return DG_EINVAL;
  if (c->host_only) {
    c->err = "context was created host-only";
    return DG_ENODEV;
  }
  if (m && c->curved.n != 0) {
    c->err = "curved elements and a learned closure do not combine";
    return DG_EINVAL;
  }
  if (m && (c->dm.N != 4 || !(norm >= 0.0) || !(p_lo >= 0.0) || !(p_hi >= p_lo) ||
            !(blend >= 0.0 && blend <= 1.0))) {
    c->err = "the learned closure needs N = 4, norm >= 0, 0 <= p_lo <= p_hi, 0 <= blend <= 1";
    return DG_EINVAL;
  }
  c->mlp = m;
  c->lbc.Wb = m ? m->Wb : nullptr;
  c->lbc.P = m ? m->P : nullptr;
  c->lbc.norm = float(norm);
  c->lbc.plo = float(p_lo);
  c->lbc.phi = float(p_hi);
  c->lbc.blend = float(blend);
  c->dm.lghost = (m && c->lbc.nl > 0) ? c->lbc.ghost : nullptr;
  drop_graphs(c);
  return DG_OK;
}

int64_t dg_learned_faces(const dg_ctx* c, int64_t* faces) {
  if (!c) return -1;
  if (faces)
    for (size_t i = 0; i < c->lface_host.size(); ++i) faces[i] = c->lface_host[i];
  return int64_t(c->lface_host.size());
}

int dg_sample_traces(dg_ctx* c, const float* q, const int64_t* faces, int64_t nf, double norm,
                     float* X, float* Y, void* stream) {
  if (!c) return DG_EINVAL;
  if (c->host_only) {
    c->err = "context was created host-only";
    return DG_ENODEV;
  }
  if (!q || !faces || !X || nf < 0 || !(norm >= 0.0)) {
    c->err = "bad argument";
    return DG_EINVAL;
  }
  const hipError_t e = dg::launch_sample_traces(c->dm, q, faces, nf, float(norm), X, Y,
                                                static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    c->err = hipGetErrorString(e);
    return DG_EHIP;
  }
  return DG_OK;
}

}  // extern "C"
