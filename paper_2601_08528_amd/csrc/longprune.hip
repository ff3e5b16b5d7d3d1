// Rank-based reordering (Sec. 5.1) of candidate lists too long for the
// one-wave LDS kernels: the reverse-edge lists of vertices that receive many
// new neighbours in one batch, and the repair and consolidation lists of
// Sec. 5.2 (alive neighbours plus entries of deleted neighbours' rows).
//
// A list's raw keys (any order, repeats allowed) sit in global memory.  The
// work runs as a chain of kernels, one workgroup per list in each, so that
// every table a kernel reads was written by an earlier launch:
//   sort    - the list's keys in LDS (bitonic), repeats removed, written back
//             in (d,id) order, with the count m of distinct candidates;
//   table   - a hash table id -> position in global memory;
//   count   - for every entry r of the row of every candidate c_j, a later
//             candidate c_i (i > j) named by it gains one detour;
//   hist    - a histogram of the detour counts;
//   select  - the threshold count tau, then the R candidates of smallest
//             (count, position), written in position order.
// The result is the same rule the LDS kernels compute, for any length up
// to kLongMaxKeys raw keys.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace svf {

namespace {

constexpr int kLongThreads = 256;

__device__ __forceinline__ const int32_t* long_row(const LongRows& rs, int32_t id) {
  return id < rs.n_old ? rs.graph + (int64_t)id * rs.R : rs.fwd + (int64_t)(id - rs.n_old) * rs.R;
}

// Inclusive sum over the 256 threads of the block (4 waves).
__device__ __forceinline__ int block_incl_sum(int v, int* sh) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int u = __shfl_up(v, o);
    if (lane >= o) v += u;
  }
  if (lane == 63) sh[wv] = v;
  __syncthreads();
  int base = 0;
  for (int i = 0; i < wv; ++i) base += sh[i];
  __syncthreads();
  return base + v;
}

__global__ __launch_bounds__(kLongThreads) void long_sort_kernel(LongLists a, int P) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int sh[4];
  uint64_t* s = reinterpret_cast<uint64_t*>(smem);
  const int l = blockIdx.x;
  const int64_t o = a.off[l];
  const int len = (int)(a.off[l + 1] - o);
  uint64_t* K = a.keys + o;
  for (int i = threadIdx.x; i < P; i += kLongThreads) s[i] = i < len ? K[i] : kKeyInf;
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += kLongThreads) {
        const int x = i ^ j;
        if (x > i) {
          const uint64_t u = s[i], v = s[x];
          const bool up = (i & k) == 0;
          if ((u > v) == up) { s[i] = v; s[x] = u; }
        }
      }
      __syncthreads();
    }
  }
  // keep the first of each run of equal keys; each thread owns a contiguous
  // segment of P / 256 positions
  const int seg = P / kLongThreads;
  const int b0 = threadIdx.x * seg;
  int mine = 0;
  for (int i = b0; i < b0 + seg; ++i)
    mine += s[i] != kKeyInf && (i == 0 || s[i] != s[i - 1]);
  const int incl = block_incl_sum(mine, sh);
  int pos = incl - mine;
  for (int i = b0; i < b0 + seg; ++i)
    if (s[i] != kKeyInf && (i == 0 || s[i] != s[i - 1])) K[pos++] = s[i];
  if (threadIdx.x == kLongThreads - 1) a.m[l] = incl;
}

__global__ __launch_bounds__(kLongThreads) void long_table_kernel(LongLists a) {
  const int l = blockIdx.x;
  const int m = a.m[l];
  if (m <= a.skip_m) return;
  const uint64_t* K = a.keys + a.off[l];
  const int64_t h0 = a.hoff[l];
  const uint32_t S = (uint32_t)((a.hoff[l + 1] - h0) / 2);
  uint32_t* tk = a.hash + h0;
  uint32_t* tv = tk + S;
  for (int i = threadIdx.x; i < m; i += kLongThreads) {
    const uint32_t id = (uint32_t)key_id(K[i]);
    uint32_t sl = slot_hash(id, S - 1u);
    for (;;) {
      if (atomicCAS(&tk[sl], kEmpty, id) == kEmpty) { tv[sl] = (uint32_t)i; break; }
      sl = (sl + 1u) & (S - 1u);
    }
  }
}

__global__ __launch_bounds__(kLongThreads) void long_count_kernel(LongLists a, LongRows rs) {
  const int l = blockIdx.x;
  const int m = a.m[l];
  if (m <= rs.R || m <= a.skip_m) return;      // every candidate is kept, or not ours
  const uint64_t* K = a.keys + a.off[l];
  const int64_t h0 = a.hoff[l];
  const uint32_t S = (uint32_t)((a.hoff[l + 1] - h0) / 2);
  const uint32_t* tk = a.hash + h0;
  const uint32_t* tv = tk + S;
  uint32_t* cnt = a.cnt + a.coff[l];
  const int R = rs.R;
  const int total = m * R;
  constexpr int kSteps = 4;                    // row entries loaded before any probe
  for (int t0 = threadIdx.x; t0 < total; t0 += kLongThreads * kSteps) {
    int32_t e[kSteps];
    int jj[kSteps];
#pragma unroll
    for (int u = 0; u < kSteps; ++u) {
      const int t = t0 + u * kLongThreads;
      jj[u] = t / R;
      e[u] = t < total ? long_row(rs, key_id(K[jj[u]]))[t - jj[u] * R] : -1;
    }
#pragma unroll
    for (int u = 0; u < kSteps; ++u) {
      if (e[u] < 0) continue;
      uint32_t sl = slot_hash((uint32_t)e[u], S - 1u);
      for (;;) {
        const uint32_t k = tk[sl];
        if (k == (uint32_t)e[u]) {
          const int i = (int)tv[sl];
          if (i > jj[u]) atomicAdd(&cnt[i], 1u);
          break;
        }
        if (k == kEmpty) break;
        sl = (sl + 1u) & (S - 1u);
      }
    }
  }
}

__global__ __launch_bounds__(kLongThreads) void long_hist_kernel(LongLists a, int R) {
  const int l = blockIdx.x;
  const int m = a.m[l];
  if (m <= R || m <= a.skip_m) return;
  const uint32_t* cnt = a.cnt + a.coff[l];
  uint32_t* hist = a.cnt + a.coff[l] + (a.off[l + 1] - a.off[l]);
  for (int i = threadIdx.x; i < m; i += kLongThreads) atomicAdd(&hist[cnt[i]], 1u);
}

__device__ __forceinline__ int wave_incl_sum(int x) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int t = __shfl_up(x, o);
    if (lane >= o) x += t;
  }
  return x;
}

__global__ __launch_bounds__(64) void long_select_kernel(LongLists a, int R, int32_t* out_ids,
                                                         float* out_d) {
  const int l = blockIdx.x;
  const int lane = lane_id();
  const int m = a.m[l];
  if (m <= a.skip_m) return;
  const uint64_t* K = a.keys + a.off[l];
  const uint32_t* cnt = a.cnt + a.coff[l];
  const uint32_t* hist = cnt + (a.off[l + 1] - a.off[l]);
  int32_t* oi = out_ids + (int64_t)a.dst[l] * R;
  float* od = out_d + (int64_t)a.dst[l] * R;
  const bool full = m > R;
  int tau = 0, need = 0;
  if (full) {
    // tau: smallest count whose cumulative frequency reaches R
    int run = 0;
    tau = -1;
    for (int c0 = 0; c0 < m && tau < 0; c0 += kWave) {
      const int h = c0 + lane < m ? (int)hist[c0 + lane] : 0;
      const int incl = wave_incl_sum(h);
      const uint64_t hit = ballot(run + incl >= R);
      if (hit) {
        const int q = __ffsll((unsigned long long)hit) - 1;
        tau = c0 + q;
        need = R - (run + __shfl(incl, q) - __shfl(h, q));
      }
      run += __shfl(incl, kWave - 1);
    }
  }
  int outpos = 0, eq_seen = 0;
  for (int c0 = 0; c0 < m && outpos < R; c0 += kWave) {
    const int i = c0 + lane;
    const bool on = i < m;
    bool sel = on;
    if (full) {
      const int c = on ? (int)cnt[i] : 0x7fffffff;
      const bool eq = on && c == tau;
      const uint64_t eb = ballot(eq);
      sel = on && (c < tau || (eq && eq_seen + lanes_below(eb) < need));
      eq_seen += popc64(eb);
    }
    const uint64_t sb = ballot(sel);
    if (sel) {
      const int p = outpos + lanes_below(sb);
      oi[p] = key_id(K[i]);
      od[p] = key_dist(K[i]);
    }
    outpos += popc64(sb);
  }
  for (int i = outpos + lane; i < R; i += kWave) { oi[i] = -1; od[i] = __builtin_inff(); }
}

}  // namespace

hipError_t launch_long_sort(const LongLists& a, int max_len, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  if (max_len > kLongMaxKeys) return hipErrorInvalidValue;
  int P = 2 * kLongThreads;
  while (P < max_len) P <<= 1;
  hipLaunchKernelGGL(long_sort_kernel, dim3(a.n), dim3(kLongThreads), (size_t)P * 8, st, a, P);
  return hipGetLastError();
}

hipError_t launch_long_prune(const LongLists& a, const LongRows& rs, int32_t* out_ids, float* out_d,
                             int64_t hash_words, int64_t cnt_words, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  hipError_t e;
  if ((e = launch_fill_u32(a.hash, hash_words, kEmpty, st)) != hipSuccess) return e;
  if ((e = launch_fill_u32(a.cnt, cnt_words, 0u, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(long_table_kernel, dim3(a.n), dim3(kLongThreads), 0, st, a);
  hipLaunchKernelGGL(long_count_kernel, dim3(a.n), dim3(kLongThreads), 0, st, a, rs);
  hipLaunchKernelGGL(long_hist_kernel, dim3(a.n), dim3(kLongThreads), 0, st, a, rs.R);
  hipLaunchKernelGGL(long_select_kernel, dim3(a.n), dim3(kWave), 0, st, a, rs.R, out_ids, out_d);
  return hipGetLastError();
}

}  // namespace svf
