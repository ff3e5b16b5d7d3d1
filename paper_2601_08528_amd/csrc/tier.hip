// Tiered vector store: in-degree counting for the placement predictor and
// the placement kernel that copies promoted rows from the host-resident store
// into HBM cache slots and updates the device mapping table (Sec. 4.2: the
// mapping h_id -> d_id | NONE; Sec. 4.3: promotion of missed vectors).
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace svf {

// E_in(x): edges pointing at x from alive vertices.
__global__ void indegree_kernel(const int32_t* __restrict__ graph, const uint32_t* __restrict__ alive,
                                int64_t n, int R, int32_t* __restrict__ e_in) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * R;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = graph[i];
    if (x >= 0 && alive_bit(alive, (int32_t)(i / R))) atomicAdd(&e_in[x], 1);
  }
}
hipError_t launch_indegree(const int32_t* graph, const uint32_t* alive, int64_t n, int R,
                           int32_t* e_in, hipStream_t st) {
  hipError_t e = launch_fill_u32(e_in, n, 0u, st);
  if (e != hipSuccess || n <= 0) return e;
  const int64_t t = n * R;
  hipLaunchKernelGGL(indegree_kernel, dim3((unsigned)std::min<int64_t>((t + 255) / 256, kMaxBlocks)),
                     dim3(256), 0, st, graph,
                     alive, n, R, e_in);
  return hipGetLastError();
}

// One workgroup per placement (slot, new id or -1, evicted id or -1): the
// row is read from the host-resident store over the host link and written to
// the cache slot, then the mapping entries of both ids are updated (a new id
// of -1 only releases the slot).  No two placements of one batch share a slot
// or an id.
__global__ void place_kernel(const int32_t* __restrict__ place, int64_t np, HostSegs store,
                             float* __restrict__ cache, int64_t stride, int32_t* __restrict__ map) {
  for (int64_t p = blockIdx.x; p < np; p += gridDim.x) {
    const int32_t slot = place[3 * p], nid = place[3 * p + 1], oid = place[3 * p + 2];
    if (nid >= 0) {
      const float* src = store.row(nid, stride);
      float* dst = cache + (int64_t)slot * stride;
      for (int64_t e = threadIdx.x; e < stride; e += blockDim.x) dst[e] = src[e];
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
      if (oid >= 0) map[oid] = -1;
      if (nid >= 0) map[nid] = slot;
    }
  }
}
hipError_t launch_place(const int32_t* place, int np, HostSegs store, float* cache,
                        int64_t stride, int32_t* map, hipStream_t st) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(place_kernel, dim3((unsigned)std::min<int64_t>(np, kMaxBlocks)), dim3(128), 0, st,
                     place, (int64_t)np, store, cache, stride, map);
  return hipGetLastError();
}

// In-degree of each cache slot's vector, in slot order: every id holding a
// slot (map[id] >= 0) writes its in-degree at that slot.  Slots no id holds
// keep what they had.
__global__ void slot_indegree_kernel(const int32_t* __restrict__ map, const int32_t* __restrict__ e_in,
                                     int64_t n, int32_t* __restrict__ sdeg) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s = map[i];
    if (s >= 0) sdeg[s] = e_in[i];
  }
}
hipError_t launch_slot_indegree(const int32_t* map, const int32_t* e_in, int64_t n, int32_t* sdeg,
                                hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, kMaxBlocks);
  hipLaunchKernelGGL(slot_indegree_kernel, dim3((unsigned)blocks), dim3(256), 0, st, map, e_in, n, sdeg);
  return hipGetLastError();
}

// Cost probe for the placement threshold (Sec. 4.3): one wave per listed
// row computes the squared L2 distance between that row and q, as a search
// gather does; the rows are the HBM cache (a hit, hs.seg null) or the host
// segments read over the host link (a miss).
__global__ __launch_bounds__(256) void probe_gather_kernel(const float* __restrict__ rows,
                                                           HostSegs hs,
                                                           const int32_t* __restrict__ idx, int n,
                                                           int64_t stride, int dim,
                                                           const float* __restrict__ q,
                                                           float* __restrict__ out) {
  const int w = (int)(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave);
  if (w >= n) return;
  const float* r = hs.seg ? hs.row(idx[w], stride) : rows + (int64_t)idx[w] * stride;
  float acc = 0.f;
  for (int e = lane_id(); e < dim; e += kWave) {
    const float d = r[e] - q[e];
    acc += d * d;
  }
  for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane_id() == 0) out[w] = acc;
}
hipError_t launch_probe_gather(const float* rows, HostSegs hs, const int32_t* idx, int n,
                               int64_t stride, int dim, const float* q, float* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(probe_gather_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, rows, hs,
                     idx, n, stride, dim, q, out);
  return hipGetLastError();
}

// Listed rows of the host segments copied into a device buffer, one
// workgroup per row, as the placement kernel copies them (also the cost
// probe of a promotion).
__global__ void gather_rows_kernel(HostSegs store, const int32_t* __restrict__ idx, int n,
                                   int64_t stride, float* __restrict__ dst) {
  for (int64_t p = blockIdx.x; p < n; p += gridDim.x) {
    const float* src = store.row(idx[p], stride);
    float* d = dst + p * stride;
    for (int64_t e = threadIdx.x; e < stride; e += blockDim.x) d[e] = src[e];
  }
}
hipError_t launch_gather_rows(HostSegs store, const int32_t* idx, int n, int64_t stride, float* dst,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)std::min<int64_t>(n, kMaxBlocks)), dim3(128),
                     0, st, store, idx, n, stride, dst);
  return hipGetLastError();
}

// Accesses of one batch: per-vertex counts, a bitmap of the vertices touched
// and (when lastpos is given) each vertex's last position in the traces
// taken in order (query, step), from nq traces of at most cap entries.
__global__ void trace_count_kernel(const int32_t* __restrict__ trace,
                                   const int32_t* __restrict__ trace_n, int nq, int cap,
                                   int32_t* __restrict__ cnt, uint32_t* __restrict__ touched,
                                   int32_t* __restrict__ lastpos) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)nq * cap) return;
  const int q = (int)(i / cap), t = (int)(i - (int64_t)q * cap);
  const int len = trace_n[q] < cap ? trace_n[q] : cap;
  if (t >= len) return;
  const int32_t x = trace[i];
  atomicAdd(&cnt[x], 1);
  atomicOr(&touched[(uint32_t)x >> 5], 1u << (x & 31));
  if (lastpos) atomicMax(&lastpos[x], (int32_t)i);
}
hipError_t launch_trace_count(const int32_t* trace, const int32_t* trace_n, int nq, int cap,
                              int32_t* cnt, uint32_t* touched, int32_t* lastpos, hipStream_t st) {
  const int64_t n = (int64_t)nq * cap;
  if (n <= 0) return hipSuccess;
  if (n > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(trace_count_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, trace,
                     trace_n, nq, cap, cnt, touched, lastpos);
  return hipGetLastError();
}

// The touched vertices of a batch in id order.  A block of 256 threads covers
// 1024 bitmap words, four per thread.  Pass 1 stores each block's number of
// touched vertices; the caller turns these into exclusive offsets; pass 2
// writes each vertex's id, access count and (when given) last position at
// its rank.
constexpr int kTouchThreads = 256;
constexpr int kTouchWordsPerThread = 4;
constexpr int64_t kTouchWordsPerBlock = (int64_t)kTouchThreads * kTouchWordsPerThread;

__global__ __launch_bounds__(256) void touched_block_count_kernel(const uint32_t* __restrict__ touched,
                                                                  int64_t words,
                                                                  int32_t* __restrict__ block_tot) {
  __shared__ int part[kTouchThreads / kWave];
  const int64_t w0 = blockIdx.x * kTouchWordsPerBlock + (int64_t)threadIdx.x * kTouchWordsPerThread;
  int c = 0;
  for (int j = 0; j < kTouchWordsPerThread; ++j)
    if (w0 + j < words) c += __popc(touched[w0 + j]);
  for (int o = kWave / 2; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if (lane_id() == 0) part[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int i = 0; i < kTouchThreads / kWave; ++i) t += part[i];
    block_tot[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(256) void touched_list_kernel(
    const uint32_t* __restrict__ touched, int64_t words, const int32_t* __restrict__ block_off,
    const int32_t* __restrict__ cnt, const int32_t* __restrict__ lastpos,
    int32_t* __restrict__ out_id, int32_t* __restrict__ out_cnt, int32_t* __restrict__ out_last) {
  __shared__ int scan[kTouchThreads];
  const int64_t w0 = blockIdx.x * kTouchWordsPerBlock + (int64_t)threadIdx.x * kTouchWordsPerThread;
  uint32_t m[kTouchWordsPerThread];
  int c = 0;
  for (int j = 0; j < kTouchWordsPerThread; ++j) {
    m[j] = w0 + j < words ? touched[w0 + j] : 0u;
    c += __popc(m[j]);
  }
  scan[threadIdx.x] = c;
  __syncthreads();
  for (int o = 1; o < kTouchThreads; o <<= 1) {
    const int v = (int)threadIdx.x >= o ? scan[threadIdx.x - o] : 0;
    __syncthreads();
    scan[threadIdx.x] += v;
    __syncthreads();
  }
  int pos = block_off[blockIdx.x] + scan[threadIdx.x] - c;
  for (int j = 0; j < kTouchWordsPerThread; ++j) {
    uint32_t w = m[j];
    while (w) {
      const int b = __ffs(w) - 1;
      w &= w - 1;
      const int32_t x = (int32_t)((w0 + j) * 32 + b);
      out_id[pos] = x;
      out_cnt[pos] = cnt[x];
      if (out_last) out_last[pos] = lastpos[x];
      ++pos;
    }
  }
}

int64_t touched_blocks(int64_t words) { return (words + kTouchWordsPerBlock - 1) / kTouchWordsPerBlock; }

hipError_t launch_touched_count(const uint32_t* touched, int64_t words, int32_t* block_tot,
                                hipStream_t st) {
  const int64_t nb = touched_blocks(words);
  if (nb <= 0) return hipSuccess;
  if (nb > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(touched_block_count_kernel, dim3((unsigned)nb), dim3(kTouchThreads), 0, st,
                     touched, words, block_tot);
  return hipGetLastError();
}

hipError_t launch_touched_list(const uint32_t* touched, int64_t words, const int32_t* block_off,
                               const int32_t* cnt, const int32_t* lastpos, int32_t* out_id,
                               int32_t* out_cnt, int32_t* out_last, hipStream_t st) {
  const int64_t nb = touched_blocks(words);
  if (nb <= 0) return hipSuccess;
  if (nb > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(touched_list_kernel, dim3((unsigned)nb), dim3(kTouchThreads), 0, st, touched,
                     words, block_off, cnt, lastpos, out_id, out_cnt, out_last);
  return hipGetLastError();
}

}  // namespace svf
