// Wave-level building blocks shared by the search and update kernels:
// LDS visited table, coalesced vector gathers with lane-group reductions,
// and the rank-based (merge path) update of a sorted key list.
#pragma once
#include "common.hpp"

namespace svf {

constexpr int kProbe = 8;
constexpr int kUnroll = 4;   // vector loads in flight per lane group

struct WaveCtx {
  uint64_t* pool;     // current pool (L keys)
  uint64_t* next;     // merge output
  uint64_t* kept;     // 64 compacted new keys
  int32_t* cid;       // 64 survivor ids
  uint32_t* vis;      // T slots
  uint32_t tmask;
  int L;
};

// ---- visited table --------------------------------------------------------
// Exact membership test (used while the table is far from full).
__device__ __forceinline__ bool vis_contains_exact(const uint32_t* vis, uint32_t mask, int32_t id) {
  uint32_t s = slot_hash((uint32_t)id, mask);
  for (;;) {
    uint32_t v = vis[s];
    if (v == (uint32_t)id) return true;
    if (v == kEmpty) return false;
    s = (s + 1) & mask;
  }
}
__device__ __forceinline__ void vis_insert_exact(uint32_t* vis, uint32_t mask, int32_t id) {
  uint32_t s = slot_hash((uint32_t)id, mask);
  for (;;) {
    uint32_t old = atomicCAS(&vis[s], kEmpty, (uint32_t)id);
    if (old == kEmpty || old == (uint32_t)id) return;
    s = (s + 1) & mask;
  }
}
// Returns true when id was seen before; otherwise records it (possibly
// overwriting another id) and returns false.
__device__ __forceinline__ bool vis_test_and_set(uint32_t* vis, uint32_t mask, int32_t id) {
  const uint32_t s0 = slot_hash((uint32_t)id, mask);
  uint32_t s = s0;
#pragma unroll 1
  for (int p = 0; p < kProbe; ++p) {
    uint32_t v = vis[s];
    if (v == (uint32_t)id) return true;
    if (v == kEmpty) {
      uint32_t old = atomicCAS(&vis[s], kEmpty, (uint32_t)id);
      if (old == kEmpty) return false;
      if (old == (uint32_t)id) return true;
    }
    s = (s + 1) & mask;
  }
  vis[s0] = (uint32_t)id;   // forget whatever lived in the first slot
  return false;
}

// ---- distances --------------------------------------------------------------
// Query slice held by each lane: NC chunks of 128 elements; within a chunk the
// lane's group covers the vector with kPer16B elements per lane.
template <typename VT, int NC>
struct QuerySlice {
  static constexpr int E = Elem<VT>::kPer16B;
  static constexpr int kLanesPerVec = 128 / E;       // 32 (FP32) or 16 (16-bit)
  static constexpr int kVecPerWave = kWave / kLanesPerVec;
  float q[NC][E];

  __device__ void load(const float* qrow, int dim, int sl) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        int idx = c * 128 + sl * E + e;
        q[c][e] = idx < dim ? Elem<VT>::round(qrow[idx]) : 0.0f;
      }
  }
};

template <typename VT, int NC>
__device__ __forceinline__ float partial_dist(const QuerySlice<VT, NC>& qs, const uint4 (&w)[NC],
                                              int metric) {
  constexpr int E = Elem<VT>::kPer16B;
  float acc = 0.0f;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    float x[E];
    Elem<VT>::unpack(w[c], x);
    if (metric == 0) {
#pragma unroll
      for (int e = 0; e < E; ++e) { float t = qs.q[c][e] - x[e]; acc = __builtin_fmaf(t, t, acc); }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) acc = __builtin_fmaf(qs.q[c][e], x[e], acc);
    }
  }
  return acc;
}

// Distances of the m (<= 64) ids in cid[] to the query; returns, in lane j,
// the key of cid[j] (kKeyInf for j >= m).
template <typename VT, int NC>
__device__ inline uint64_t gather_keys(const QuerySlice<VT, NC>& qs, const VT* __restrict__ base,
                                int64_t stride, const int32_t* cid, int m, int metric) {
  using QS = QuerySlice<VT, NC>;
  constexpr int E = QS::E;
  constexpr int LPV = QS::kLanesPerVec;
  constexpr int VPW = QS::kVecPerWave;
  const int lane = lane_id();
  const int sub = lane / LPV, sl = lane % LPV;
  float mine = 0.0f;
  const int steps = (m + VPW - 1) / VPW;
  for (int s0 = 0; s0 < steps; s0 += kUnroll) {
    uint4 w[kUnroll][NC];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int j = (s0 + u) * VPW + sub;
      const bool on = (s0 + u) < steps && j < m;
      const int32_t id = on ? cid[j] : 0;
      const VT* row = base + (int64_t)id * stride;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int off = c * 128 + sl * E;
        if (on && off < stride)
          w[u][c] = *reinterpret_cast<const uint4*>(row + off);
        else
          w[u][c] = make_uint4(0, 0, 0, 0);
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      float acc = partial_dist<VT, NC>(qs, w[u], metric);
#pragma unroll
      for (int o = LPV / 2; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
      // vector j = step * VPW + slot lives in lanes [slot*LPV, slot*LPV+LPV)
      const float got = __shfl(acc, (lane % VPW) * LPV);
      if (lane / VPW == s0 + u) mine = got;
    }
  }
  if (lane >= m) return kKeyInf;
  const float d = metric == 0 ? mine : -mine;
  return make_key(d, cid[lane]);
}

// ---- pool merge ---------------------------------------------------------------
// Merge one sorted key per lane (kKeyInf padded) into the sorted pool of L
// keys, keeping the L smallest; keys equal in (dist,id) to a pool entry are
// dropped (the pool entry keeps its expanded flag).
__device__ inline void merge_into_pool(WaveCtx& w, uint64_t nk) {
  const int lane = lane_id();
  const int L = w.L;
  const uint64_t* cur = w.pool;
  int lo = L;
  bool keep = false;
  if (nk != kKeyInf) {
    const uint64_t o = key_ord(nk);
    int a = 0, b = L;
    while (a < b) {                      // first pool key not below nk
      int mid = (a + b) >> 1;
      if (key_ord(cur[mid]) < o) a = mid + 1; else b = mid;
    }
    lo = a;
    const bool dup = lo < L && key_ord(cur[lo]) == o;
    keep = !dup && lo < L;
  }
  const uint64_t kb = ballot(keep);
  const int r = lanes_below(kb);
  const int mk = popc64(kb);
  if (keep) w.kept[r] = nk;
  __syncthreads();
  if (mk == 0) return;
  if (keep && r + lo < L) w.next[r + lo] = nk;
  for (int i = lane; i < L; i += kWave) {
    const uint64_t pk = cur[i];
    const uint64_t o = key_ord(pk);
    int a = 0, b = mk;                   // kept keys below this pool key
    while (a < b) {
      int mid = (a + b) >> 1;
      if (key_ord(w.kept[mid]) < o) a = mid + 1; else b = mid;
    }
    if (i + a < L) w.next[i + a] = pk;
  }
  __syncthreads();
  uint64_t* t = w.pool; w.pool = w.next; w.next = t;
}


}  // namespace svf
