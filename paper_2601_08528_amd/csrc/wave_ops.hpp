// Wave-level building blocks shared by the search and update kernels:
// LDS visited table, coalesced vector gathers with lane-group reductions,
// and the rank-based (merge path) update of a sorted key list.
#pragma once
#include "common.hpp"
#include "kernels.hpp"

namespace svf {

constexpr int kProbe = 8;

struct WaveCtx {
  uint64_t* pool;     // current pool (L keys)
  uint64_t* next;     // merge output
  uint64_t* kept;     // 64 compacted new keys
  int32_t* cid;       // 64 survivor ids
  uint32_t* vis;      // T slots
  uint32_t tmask;
  int L;
  int ktrack;         // report merges that change the first ktrack keys (0: off)
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

// ---- visited tables ----------------------------------------------------------
// Both policies answer "seen before?" without false positives and may forget
// (the search result does not depend on forgetting, only the work does).
//
// VisLinear32: 32-bit ids, open addressing with a bounded probe run; on a
// full run the first slot is overwritten.
struct VisLinear32 {
  uint32_t* t;
  uint32_t mask;
  __device__ static size_t bytes(int T) { return (size_t)T * 4; }
  __device__ void setup(void* p, int T, int /*id_bits*/) {
    t = static_cast<uint32_t*>(p);
    mask = (uint32_t)T - 1u;
  }
  __device__ void clear(int T) {
    for (int i = lane_id(); i < T; i += kWave) t[i] = kEmpty;
  }
  __device__ bool test_and_set(int32_t id) { return vis_test_and_set(t, mask, id); }
};

// VisTags: ids below 2^B are scrambled by a bijection of [0, 2^B)
// (multiplication by an odd constant modulo 2^B); the high bits pick a set,
// the low bits are the tag, so a tag match identifies the id exactly.  Tags
// are packed: 12-bit fields, five to a 64-bit set, when tag_bits <= 11, else
// 16-bit fields, four to a set (needs B - log2(sets) <= 15).  A new id enters a
// set by shifting the set word up one field, so the oldest id of a full set
// is the one forgotten (ids seen early in a search lie farthest from where
// it ends).  Lanes that race on one set can only lose insertions; every tag a
// set holds was inserted, so the table still never reports an unseen id.
// A tag is found without a loop: the set word XOR the tag copied into every
// field has a zero field exactly when some field holds the tag, which the
// borrow test (x - ones) & ~x & highs detects (a borrow can only start at a
// zero field, so it reports no field that is not zero).
struct VisTags {
  uint64_t* sets;
  uint32_t idmask;
  int tag_bits, fb;
  uint64_t keep, ones, highs;
  __device__ void setup(void* p, int T, int id_bits) {
    sets = static_cast<uint64_t*>(p);
    const int set_bits = 31 - __clz(T / 4);
    idmask = id_bits >= 32 ? 0xffffffffu : ((1u << id_bits) - 1u);
    tag_bits = id_bits - set_bits;
    fb = tag_bits <= 11 ? 12 : 16;
    keep = fb == 12 ? ((1ull << 60) - 1ull) : ~0ull;
    ones = fb == 12 ? 0x001001001001001ull : 0x0001000100010001ull;
    highs = ones << (fb - 1);
  }
  __device__ void clear(int T) {
    for (int i = lane_id(); i < T / 4; i += kWave) sets[i] = 0ull;
  }
  __device__ bool test_and_set(int32_t id) {
    const uint32_t h = ((uint32_t)id * 0x9E3779B1u) & idmask;
    const uint32_t set = h >> tag_bits;
    const uint64_t tag = (uint64_t)((h & ((1u << tag_bits) - 1u)) + 1u);
    const uint64_t w = sets[set];
    const uint64_t x = w ^ (tag * ones);
    if (((x - ones) & ~x & highs) != 0ull) return true;
    sets[set] = ((w << fb) | tag) & keep;
    return false;
  }
};

// ---- distances --------------------------------------------------------------
// Query slice held by each lane: NC chunks of 128 elements; within a chunk the
// lane's group covers the vector with kPer16B elements per lane.
template <typename VT, int NC>
struct QuerySlice {
  static constexpr int E = Elem<VT>::kPer16B;
  static constexpr int kLanesPerVec = 128 / E;       // 32 (FP32) or 16 (16-bit)
  static constexpr int kVecPerWave = kWave / kLanesPerVec;
  float q[NC][E];

  // All lanes of the wave call load; the lanes of one group hold one copy of
  // the query between them.  The FP8 form quantises the query like a stored
  // vector (its own scale, E4M3 codes) and keeps the FP32 products s * value.
  __device__ void load(const float* qrow, int dim, int sl) {
    if constexpr (Elem<VT>::kScaled) {
      float m = 0.0f;
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int idx = c * 128 + sl * E + e;
          q[c][e] = idx < dim ? qrow[idx] : 0.0f;
          m = __builtin_fmaxf(m, __builtin_fabsf(q[c][e]));
        }
#pragma unroll
      for (int o = 1; o < kLanesPerVec; o <<= 1) m = __builtin_fmaxf(m, __shfl_xor(m, o));
      const float s = fp8_scale_of(m);
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int e = 0; e < E; ++e)
          q[c][e] = __fmul_rn(s, Elem<VT>::value(f32_to_e4m3_sat(__fdiv_rn(q[c][e], s))));
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int e = 0; e < E; ++e) {
          int idx = c * 128 + sl * E + e;
          q[c][e] = idx < dim ? Elem<VT>::round(qrow[idx]) : 0.0f;
        }
    }
  }
};

// Partial distance over the lane's slice.  A scaled (FP8) vector stands for
// xs * value(code): for L2 each difference q - xs * value is formed by one
// fused multiply-add; for the inner product the sum of q * value is returned
// and the caller multiplies the whole sum by xs.
template <typename VT, int NC>
__device__ __forceinline__ float partial_dist(const QuerySlice<VT, NC>& qs, const uint4 (&w)[NC],
                                              int metric, float xs = 1.0f) {
  constexpr int E = Elem<VT>::kPer16B;
  float acc = 0.0f;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    float x[E];
    Elem<VT>::unpack(w[c], x);
    if (metric == 0) {
      if constexpr (Elem<VT>::kScaled) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const float t = __builtin_fmaf(-xs, x[e], qs.q[c][e]);
          acc = __builtin_fmaf(t, t, acc);
        }
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) { float t = qs.q[c][e] - x[e]; acc = __builtin_fmaf(t, t, acc); }
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) acc = __builtin_fmaf(qs.q[c][e], x[e], acc);
    }
  }
  return acc;
}

// Sum of U per-lane partials across each group of LPV lanes, as a
// reduce-scatter: every stage halves the values a lane holds and exchanges the
// other half with its partner, so U sums need about U + log2(LPV) shuffles
// instead of U * log2(LPV).  Each pairwise addition combines the same two
// subtrees as a plain butterfly would, so every sum is bitwise the value a
// butterfly reduction gives, whatever its position in the batch.  Lane l of a
// group ends with the sum of step l / (LPV / U).
template <int LPV, int U, int S = 0>
__device__ __forceinline__ void reduce_scatter_stage(float (&acc)[U], int lane) {
  if constexpr ((U >> S) > 1) {
    constexpr int o = LPV >> (S + 1);
    constexpr int half = (U >> S) / 2;
    const bool hi = (lane & o) != 0;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      // select values, not array elements: a conditional over two elements
      // is an address select, which keeps acc in scratch memory
      const float lo_v = acc[i], hi_v = acc[i + half];
      const float send = hi ? lo_v : hi_v;
      const float keep = hi ? hi_v : lo_v;
      acc[i] = keep + xor_lane_f<o>(send);
    }
    reduce_scatter_stage<LPV, U, S + 1>(acc, lane);
  }
}
template <int O>
__device__ __forceinline__ float butterfly_down(float r) {
  if constexpr (O >= 1) {
    r += xor_lane_f<O>(r);
    return butterfly_down<O / 2>(r);
  } else {
    return r;
  }
}
template <int LPV, int U>
__device__ __forceinline__ float reduce_scatter(float (&acc)[U]) {
  reduce_scatter_stage<LPV, U>(acc, lane_id());
  return butterfly_down<LPV / U / 2>(acc[0]);
}

// Vector steps gathered per round trip, powers of two, fewer for wider
// vectors: FP32 16 steps of 2 vectors (32 vectors of one 128-element chunk),
// 16-bit 8 steps of 4 on full rows and 4 steps on short ones, FP8 4 steps of
// 8.  Chosen by measurement on 1M-vector indexes of 128 and 96 dimensions;
// more steps in flight only cost registers there.
#ifndef SVF_GATHER_STEPS_F32
#define SVF_GATHER_STEPS_F32 16
#endif
#ifndef SVF_GATHER_STEPS_16
#define SVF_GATHER_STEPS_16 4
#endif
#ifndef SVF_GATHER_STEPS_16_FULL
#define SVF_GATHER_STEPS_16_FULL 8
#endif
#ifndef SVF_GATHER_STEPS_8
#define SVF_GATHER_STEPS_8 4
#endif
template <typename VT, int NC, int FORM> struct GatherSteps {
  static constexpr int base = sizeof(VT) == 4   ? SVF_GATHER_STEPS_F32
                              : sizeof(VT) == 2 ? (FORM == 2 ? SVF_GATHER_STEPS_16_FULL
                                                             : SVF_GATHER_STEPS_16)
                                                : SVF_GATHER_STEPS_8;
  // at least two steps, except one for eight chunks: there the 16-bit and
  // FP8 query slices and two steps of loads spilled (768 dimensions, BF16:
  // 5.5 -> 4.0 ms per 10k queries with one step)
  static constexpr int value = base / NC >= 2 ? base / NC : (NC >= 8 ? 1 : 2);
};

// The distance rounds of gather_keys: returns, in lane j < m, the summed
// distance of candidate j.  FORM 0: each lane loads only its own candidate's
// slice (predicated); FORM 1: lanes past m load candidate 0's row instead,
// only the slices past a short row are predicated; FORM 2: as 1, for rows
// whose every 16-byte slice lies inside (stride >= NC * 128 elements), with
// no per-lane test at all.  The tiered variant is always FORM 0.
template <typename VT, int NC, bool TIER, int FORM>
__device__ inline float gather_rounds(const QuerySlice<VT, NC>& qs, const VT* __restrict__ base,
                                      int64_t stride, const int32_t* cid, int m, int metric,
                                      const int32_t* slot, const VT* __restrict__ tcache,
                                      const float* __restrict__ vscale, HostSegs hs,
                                      const float* vj) {
  constexpr bool kScaled = Elem<VT>::kScaled;
  using QS = QuerySlice<VT, NC>;
  constexpr int E = QS::E;
  constexpr int LPV = QS::kLanesPerVec;
  constexpr int VPW = QS::kVecPerWave;
  // the tiered variant keeps half as many loads in flight (its row choice
  // needs registers); the reduction tree, and so every sum, is the same
  constexpr int kSteps = GatherSteps<VT, NC, FORM>::value;
  constexpr int UB = kSteps < LPV ? kSteps : LPV;
  constexpr int U = TIER ? (UB / 2 < 2 ? 2 : UB / 2) : UB;
  // the reduction hands whole lane groups down: U must be a power of two
  // that divides LPV
  static_assert(U >= 1 && (U & (U - 1)) == 0 && LPV % U == 0, "gather steps");
  const int lane = lane_id();
  const int sub = lane / LPV, sl = lane % LPV;
  const uint32_t ustride = (uint32_t)stride;
  float mine = 0.0f;
  const int steps = (m + VPW - 1) / VPW;
  for (int s0 = 0; s0 < steps; s0 += U) {
    uint4 w[U][NC];
    float xs[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = (s0 + u) * VPW + sub;
      const bool on = j < m;
      if constexpr (TIER) {
        const int32_t id = on ? cid[j] : 0;
        const VT* row = hs.seg ? reinterpret_cast<const VT*>(hs.row(id, stride))
                               : base + (uint64_t)(uint32_t)id * ustride;
        if constexpr (kScaled) xs[u] = on ? vscale[id] : 0.0f;
        else xs[u] = 1.0f;
        const int32_t sl_ = on && slot ? slot[j] : -1;
        if (sl_ >= 0) row = tcache + (uint64_t)(uint32_t)sl_ * ustride;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int off = c * 128 + sl * E;
          if (on && off < stride)
            w[u][c] = *reinterpret_cast<const uint4*>(row + off);
          else
            w[u][c] = make_uint4(0, 0, 0, 0);
        }
      } else if constexpr (FORM != 0) {
        // lanes past m read candidate 0's row (its own lanes load it too);
        // their sums stay in their own lane group and are dropped later
        const int32_t id = cid[on ? j : 0];
        const VT* row = base + (uint64_t)(uint32_t)id * ustride;
        if constexpr (kScaled) xs[u] = vscale[id];
        else xs[u] = 1.0f;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int off = c * 128 + sl * E;
          if (FORM == 2 || off < stride)
            w[u][c] = *reinterpret_cast<const uint4*>(row + off);
          else
            w[u][c] = make_uint4(0, 0, 0, 0);
        }
      } else {
        const int32_t id = on ? cid[j] : 0;
        const VT* row = base + (uint64_t)(uint32_t)id * ustride;
        if constexpr (kScaled) xs[u] = on ? (vj ? vj[j] : vscale[id]) : 0.0f;
        else xs[u] = 1.0f;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int off = c * 128 + sl * E;
          if (on && off < stride)
            w[u][c] = *reinterpret_cast<const uint4*>(row + off);
          else
            w[u][c] = make_uint4(0, 0, 0, 0);
        }
      }
    }
    float acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = partial_dist<VT, NC>(qs, w[u], metric, xs[u]);
    const float r = reduce_scatter<LPV, U>(acc);
    // lane j takes vector j = (s0 + u) * VPW + h from lane h * LPV + u * (LPV / U)
    const int u = lane / VPW - s0;
    const int h = lane % VPW;
    const int src = h * LPV + ((u >= 0 && u < U) ? u : 0) * (LPV / U);
    const float got = __shfl(r, src);
    if (u >= 0 && u < U) mine = got;
  }
  return mine;
}

// Distances of the m (<= 64) ids in cid[] to the query; returns, in lane j,
// the key of cid[j] (kKeyInf for j >= m).  A step gathers VPW vectors, one per
// group of LPV lanes; U steps are loaded before any is consumed.  FORM picks
// the load rounds of gather_rounds; every form gives the same sums.  Forms 1
// and 2 are for unscaled, untiered stores, and form 2 needs stride >= NC * 128.
// A kernel inlines one form only: with two, the compiler keeps the step arrays
// in scratch memory.
// With a tier (TIER), vector j is read from tcache row slot[j] when that slot
// is >= 0 (slot may be null: no cache) and otherwise from row cid[j] of the
// host segments hs, or of base when hs has none.  A scaled (FP8) store reads the
// vector's scale from vscale[id] with its row, or, when vj is given, takes
// candidate j's scale from vj[j] (the scales a row carries beside its ids).
template <typename VT, int NC, bool TIER = false, int FORM = 0>
__device__ inline uint64_t gather_keys(const QuerySlice<VT, NC>& qs, const VT* __restrict__ base,
                                       int64_t stride, const int32_t* cid, int m, int metric,
                                       const int32_t* slot = nullptr,
                                       const VT* __restrict__ tcache = nullptr,
                                       const float* __restrict__ vscale = nullptr,
                                       HostSegs hs = HostSegs{nullptr, 0},
                                       const float* vj = nullptr) {
  constexpr bool kScaled = Elem<VT>::kScaled;
  static_assert(FORM == 0 || (!TIER && !kScaled), "gather form");
  const int lane = lane_id();
  const float mine = gather_rounds<VT, NC, TIER, FORM>(qs, base, stride, cid, m, metric, slot,
                                                       tcache, vscale, hs, vj);
  if (lane >= m) return kKeyInf;
  float x = mine;
  if (kScaled && metric != 0) x *= vj ? vj[lane] : vscale[cid[lane]];
  const float d = metric == 0 ? x : -x;
  return make_key(d, cid[lane]);
}

// ---- pool merge ---------------------------------------------------------------
// Merge one sorted key per lane (kKeyInf padded) into the sorted pool of L
// keys, keeping the L smallest; keys equal in (dist,id) to a pool entry are
// dropped (the pool entry keeps its expanded flag).
template <class S = BlockSync>
__device__ inline bool merge_into_pool(WaveCtx& w, uint64_t nk) {
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
  S::sync();
  if (mk == 0) return false;
  const bool topk = ballot(keep && r + lo < w.ktrack) != 0;
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
  S::sync();
  uint64_t* t = w.pool; w.pool = w.next; w.next = t;
  return topk;
}


// Ascending bitonic sort of the keys held by the first W lanes (W a power of
// two); the other lanes must hold kKeyInf.  (A fully unrolled form with
// constant exchange distances measured slower: its code grows with every
// width it must cover.)
__device__ __forceinline__ uint64_t wave_sort_width(uint64_t key, int W) {
  const int lane = lane_id();
  for (int k = 2; k <= W; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      const uint64_t other = __shfl_xor(key, j);
      const bool up = (lane & k) == 0;
      const bool low = (lane & j) == 0;
      const uint64_t mn = key < other ? key : other;
      const uint64_t mx = key < other ? other : key;
      key = (low == up) ? mn : mx;
    }
  }
  return key;
}

// Merge one unsorted key per lane (kKeyInf = none) into the pool: keys that
// cannot enter a full pool are dropped first, the rest are compacted and
// sorted over the narrowest power-of-two width, then merged.
template <class S = BlockSync>
__device__ inline bool sort_merge(WaveCtx& w, uint64_t k) {
  const int lane = lane_id();
  const uint64_t last = w.pool[w.L - 1];
  const bool live = k != kKeyInf && (last == kKeyInf || key_ord(k) < key_ord(last));
  const uint64_t lb = ballot(live);
  const int s = popc64(lb);
  if (s == 0) return false;
  S::sync();
  if (live) w.kept[lanes_below(lb)] = k;
  S::sync();
  uint64_t c = lane < s ? w.kept[lane] : kKeyInf;
  int W = 1;
  while (W < s) W <<= 1;
  c = wave_sort_width(c, W);
  S::sync();
  return merge_into_pool<S>(w, c);
}

}  // namespace svf
