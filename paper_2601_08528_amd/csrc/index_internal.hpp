// Internal helpers of the index shared by the C ABI (index.hip) and the
// serving runtime (serve.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "index.hpp"
#include "kernels.hpp"

namespace svf_detail {

int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define CK(call)                                         \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return svf_detail::hip_fail(e_, #call); \
  } while (0)

template <class T>
int scratch(svf::DevBuf& b, size_t count, T** out) {
  hipError_t e = b.ensure(count * sizeof(T) + 16);
  if (e != hipSuccess) return hip_fail(e, "scratch allocation");
  *out = b.as<T>();
  return SVF_OK;
}
// The same for buffers sized by counts that vary from call to call: a
// reallocation leaves an eighth more room, so that slowly growing counts do
// not reallocate (and synchronize the device) on every call.
template <class T>
int scratch_grow(svf::DevBuf& b, size_t count, T** out) {
  const size_t need = count * sizeof(T) + 16;
  hipError_t e = b.ensure(need, need + need / 8);
  if (e != hipSuccess) return hip_fail(e, "scratch allocation");
  *out = b.as<T>();
  return SVF_OK;
}

struct PendingInsert {
  bool seed = false;
  int64_t n0 = 0, b = 0;
  int n_targets = 0;
  svf::ReverseArgs ra{};
};

int reserve(svf_index* ix, int64_t need);
int insert_prepare(svf_index* ix, const float* d_vecs, int64_t b, PendingInsert* p);
int insert_commit(svf_index* ix, PendingInsert* p);
int repair(svf_index* ix, int consolidate);
int delete_ids(svf_index* ix, const int32_t* ids, int64_t n);
int bg_merge(svf_index* ix);
svf::SearchArgs base_args(const svf_index* ix);
void set_beam(svf::SearchArgs& a, const svf_index* ix, int L);
int check_search_args(const svf_index* ix, int64_t nq, int k, int beam);
// Search of nq device-resident queries on stream st.  ws_qkey (nq words of
// device memory) replaces the index's own key buffer when given; the batch
// totals are then not kept, and the learned form and the tiered store, which
// need more workspace, are refused.
int search_impl(svf_index* ix, const float* d_q, int64_t nq, int k, int beam, int32_t* d_ids,
                float* d_d, int32_t* d_nd, int32_t* d_ne, hipStream_t st,
                uint64_t* ws_qkey = nullptr);
bool all_finite(const float* p, int64_t n);
// The search of nq device-resident queries with CPU-GPU co-processing of the
// tiered store's misses (FP32 traversal, random entry points); `a` is the
// filled argument block of the one-kernel search.
int co_search(svf_index* ix, const svf::SearchArgs& a, const float* d_q, int64_t nq, hipStream_t st);
// Host-core nanoseconds per distance of that path over the rows ids[0..n).
double host_distance_ns(svf_index* ix, const int32_t* ids, int n);
int beam_insert(const svf_index* ix);
void serve_shutdown(svf_index* ix);

}  // namespace svf_detail
