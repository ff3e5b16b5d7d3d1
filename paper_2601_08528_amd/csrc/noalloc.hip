// Search that allocates no device memory (svf_search_dev_noalloc).
//
// The search's only per-call device workspace is one 64-bit entry-stream key
// per query.  Here it lives in `scratch`, a fixed array of device memory that
// each GPU holds from the load of the library to the end of the process.  In
// host code the array's name does not denote device memory: its address on a
// device is taken once per device with hipGetSymbolAddress (with that device
// current) and kept in g_scratch; kernels receive that pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "index.hpp"
#include "index_internal.hpp"
#include "svf.h"

namespace {

constexpr int64_t kNoAllocMaxQueries = 1 << 19;               // 524,288 queries
constexpr size_t kScratchBytes = (size_t)kNoAllocMaxQueries * 8;  // 4 MiB

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on `dev`, taken once per device.
int scratch_on(int dev, void** out) {
  using svf_detail::fail;
  if (dev < 0 || dev >= kMaxDevices) return fail(SVF_E_DEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_scratch[dev]) {
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return fail(SVF_E_DEVICE, "hipGetDevice failed");
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return fail(SVF_E_DEVICE, "hipSetDevice failed");
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) return svf_detail::hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return SVF_OK;
}

}  // namespace

extern "C" int svf_search_dev_noalloc(svf_index* ix, const float* d_queries, int64_t nq, int32_t k,
                                      int32_t beam, int32_t* d_out_ids, float* d_out_dists,
                                      int32_t* d_n_dist, int32_t* d_n_exp, void* stream) {
  using svf_detail::fail;
  if (ix && ix->server) return fail(SVF_E_BUSY, "index is serving: use svf_submit_search");
  int rc = svf_detail::check_search_args(ix, nq, k, beam);
  if (rc) return rc;
  if (nq > kNoAllocMaxQueries)
    return fail(SVF_E_INVAL, "svf_search_dev_noalloc: nq above 524288 (its fixed workspace)");
  if (ix->opt.use_model && ix->model)
    return fail(SVF_E_INVAL, "svf_search_dev_noalloc: the learned form (use_model) needs svf_search_dev");
  if (ix->tier.on)
    return fail(SVF_E_INVAL, "svf_search_dev_noalloc: a tiered store needs svf_search_dev");
  if (nq > 0 && (!d_queries || !d_out_ids || !d_out_dists)) return fail(SVF_E_INVAL, "null buffer");
  if (nq == 0) return SVF_OK;
  void* ws = nullptr;
  if ((rc = scratch_on(ix->device, &ws))) return rc;
  std::lock_guard<std::mutex> g(ix->mu);
  return svf_detail::search_impl(ix, d_queries, nq, k, beam, d_out_ids, d_out_dists, d_n_dist,
                                 d_n_exp, (hipStream_t)stream, static_cast<uint64_t*>(ws));
}
