// C ABI of the standalone entry/stop predictor (the network an index trains
// in svf_model_fit), exposed so its forward pass, gradients and training can
// be checked on their own.
#include <hip/hip_runtime.h>

#include <new>
#include <string>

#include "../../include/svf.h"
#include "mlp.hpp"

struct svf_mlp {
  svf::Mlp* m = nullptr;
  hipStream_t st = nullptr;
  void* buf = nullptr;   // staging for host-pointer calls
  size_t buf_bytes = 0;
};

namespace {
thread_local std::string g_merr;
int mfail(int code, const std::string& msg) {
  g_merr = msg;
  return code;
}
#define MCK_ABI(call)                                                            \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess)                                                        \
      return mfail(e_ == hipErrorOutOfMemory ? SVF_E_NOMEM : SVF_E_DEVICE,       \
                   std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

int stage(svf_mlp* m, size_t bytes, char** out) {
  if (bytes > m->buf_bytes) {
    if (m->buf) (void)hipFree(m->buf);
    m->buf = nullptr;
    m->buf_bytes = 0;
    if (hipMalloc(&m->buf, bytes) != hipSuccess) return mfail(SVF_E_NOMEM, "staging allocation");
    m->buf_bytes = bytes;
  }
  *out = static_cast<char*>(m->buf);
  return SVF_OK;
}
}  // namespace

extern "C" {

const char* svf_mlp_last_error(void) { return g_merr.c_str(); }

int svf_mlp_create(int32_t din, int32_t hidden, int32_t n_clusters, uint64_t seed, svf_mlp** out) {
  if (!out) return mfail(SVF_E_INVAL, "null output");
  *out = nullptr;
  if (din < 1 || din > 1024 || hidden < 1 || hidden > 4096 || n_clusters < 2 || n_clusters > 1024)
    return mfail(SVF_E_INVAL, "bad predictor dimensions");
  svf_mlp* m = new (std::nothrow) svf_mlp();
  if (!m) return mfail(SVF_E_NOMEM, "host allocation");
  m->m = new (std::nothrow) svf::Mlp(din, hidden, n_clusters, seed);
  hipError_t e;
  if (!m->m || (e = hipStreamCreateWithFlags(&m->st, hipStreamNonBlocking)) != hipSuccess ||
      (e = m->m->init_device(m->st)) != hipSuccess) {
    svf_mlp_destroy(m);
    return mfail(SVF_E_DEVICE, "predictor setup");
  }
  *out = m;
  return SVF_OK;
}

int svf_mlp_destroy(svf_mlp* m) {
  if (!m) return SVF_OK;
  if (m->st) (void)hipStreamSynchronize(m->st);
  delete m->m;
  if (m->buf) (void)hipFree(m->buf);
  if (m->st) (void)hipStreamDestroy(m->st);
  delete m;
  return SVF_OK;
}

int svf_mlp_num_params(const svf_mlp* m, int64_t* n) {
  if (!m || !n) return mfail(SVF_E_INVAL, "null argument");
  *n = m->m->dims().total();
  return SVF_OK;
}

int svf_mlp_set_params(svf_mlp* m, const float* params) {
  if (!m || !params) return mfail(SVF_E_INVAL, "null argument");
  MCK_ABI(m->m->set_params(params, m->st));
  return SVF_OK;
}

int svf_mlp_get_params(const svf_mlp* cm, float* params) {
  if (!cm || !params) return mfail(SVF_E_INVAL, "null argument");
  svf_mlp* m = const_cast<svf_mlp*>(cm);
  MCK_ABI(m->m->get_params(params, m->st));
  return SVF_OK;
}

int svf_mlp_forward(svf_mlp* m, const float* x, int64_t n, float* out) {
  if (!m || (n > 0 && (!x || !out)) || n < 0) return mfail(SVF_E_INVAL, "bad argument");
  if (n == 0) return SVF_OK;
  const svf::MlpDims& d = m->m->dims();
  char* b;
  int rc = stage(m, (size_t)n * (d.din + d.no()) * 4, &b);
  if (rc) return rc;
  float* dx = reinterpret_cast<float*>(b);
  float* dz = dx + n * d.din;
  MCK_ABI(hipMemcpyAsync(dx, x, (size_t)n * d.din * 4, hipMemcpyHostToDevice, m->st));
  MCK_ABI(m->m->forward(dx, n, dz, m->st));
  MCK_ABI(hipMemcpyAsync(out, dz, (size_t)n * d.no() * 4, hipMemcpyDeviceToHost, m->st));
  MCK_ABI(hipStreamSynchronize(m->st));
  return SVF_OK;
}

int svf_mlp_loss_grad(svf_mlp* m, const float* x, const int32_t* label, const float* log_stop,
                      int64_t n, float lambda, float delta, float* loss, float* grad) {
  if (!m || !x || !label || !log_stop || !grad || n < 1) return mfail(SVF_E_INVAL, "bad argument");
  const svf::MlpDims& d = m->m->dims();
  for (int64_t i = 0; i < n; ++i)
    if (label[i] < 0 || label[i] >= d.nc) return mfail(SVF_E_INVAL, "label out of range");
  char* b;
  const int64_t np = d.total();
  int rc = stage(m, (size_t)(n * d.din + n + n + np) * 4, &b);
  if (rc) return rc;
  float* dx = reinterpret_cast<float*>(b);
  int32_t* dl = reinterpret_cast<int32_t*>(dx + n * d.din);
  float* ds = reinterpret_cast<float*>(dl + n);
  float* dg = ds + n;
  MCK_ABI(hipMemcpyAsync(dx, x, (size_t)n * d.din * 4, hipMemcpyHostToDevice, m->st));
  MCK_ABI(hipMemcpyAsync(dl, label, (size_t)n * 4, hipMemcpyHostToDevice, m->st));
  MCK_ABI(hipMemcpyAsync(ds, log_stop, (size_t)n * 4, hipMemcpyHostToDevice, m->st));
  float l = 0.f;
  MCK_ABI(m->m->loss_grad(dx, dl, ds, n, lambda, delta, dg, &l, m->st));
  MCK_ABI(hipMemcpyAsync(grad, dg, (size_t)np * 4, hipMemcpyDeviceToHost, m->st));
  MCK_ABI(hipStreamSynchronize(m->st));
  if (loss) *loss = l;
  return SVF_OK;
}

int svf_mlp_train(svf_mlp* m, const float* x, const int32_t* label, const float* log_stop,
                  int64_t n, int32_t epochs, int32_t batch, float lr, float lambda, float delta,
                  float* last_loss) {
  if (!m || !x || !label || !log_stop || n < 1 || epochs < 1 || batch < 1 || batch > n)
    return mfail(SVF_E_INVAL, "bad argument");
  const svf::MlpDims& d = m->m->dims();
  for (int64_t i = 0; i < n; ++i)
    if (label[i] < 0 || label[i] >= d.nc) return mfail(SVF_E_INVAL, "label out of range");
  char* b;
  int rc = stage(m, (size_t)(n * d.din + n + n) * 4, &b);
  if (rc) return rc;
  float* dx = reinterpret_cast<float*>(b);
  int32_t* dl = reinterpret_cast<int32_t*>(dx + n * d.din);
  float* ds = reinterpret_cast<float*>(dl + n);
  MCK_ABI(hipMemcpyAsync(dx, x, (size_t)n * d.din * 4, hipMemcpyHostToDevice, m->st));
  MCK_ABI(hipMemcpyAsync(dl, label, (size_t)n * 4, hipMemcpyHostToDevice, m->st));
  MCK_ABI(hipMemcpyAsync(ds, log_stop, (size_t)n * 4, hipMemcpyHostToDevice, m->st));
  MCK_ABI(m->m->train(dx, dl, ds, n, epochs, batch, lr, lambda, delta, last_loss, m->st));
  return SVF_OK;
}

}  // extern "C"
