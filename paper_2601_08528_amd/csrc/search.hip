// Batched best-first graph search (SVFusion, Sec. 4.2, Algorithm 1) on one
// device tier, one wavefront per query.
//
// Per query the wave keeps in LDS
//   - the candidate pool: `L` sorted 64-bit keys (dist, id, expanded flag),
//     double-buffered so a merge writes the next pool while reading this one;
//   - a visited table: exact tags of the ids in small sets, the oldest of a
//     full set forgotten (or, for ids too wide for tags, 32-bit ids with a
//     bounded probe run).  The table may forget ids but never reports an
//     unvisited id as visited.  Forgetting costs only repeated distance
//     evaluations: an id that left the pool had L smaller keys, the L-th key
//     never grows, so it is rejected again, and an id still in the pool is
//     recognised by its identical key during the merge.  During the entry
//     phase the table's LDS holds an exact list of the accepted entries.
//
// One iteration: the smallest unexpanded key is the parent (Algorithm 1,
// GetNearest); its row of R ids is read with one coalesced load; ids that are
// INVALID, deleted (bitset) or visited are dropped; the survivors are compacted
// and their vectors gathered so that each 8-lane (FP8), 16-lane (16-bit) or
// 32-lane (FP32) group reads one 128/256/512-byte vector with 16-byte loads; the
// group reduces its partial sums by lane shuffles; the new keys are sorted
// across the wave (bitonic) and merged into the pool by rank (merge path),
// which also drops re-evaluated ids.  The loop ends when every pool entry is
// expanded (or after max_iters expansions).
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"
#include "wave_ops.hpp"

namespace svf {

// ---------------------------------------------------------------------------
template <typename VT, int NC, typename VIS, bool TIER, bool FULL>
__global__ __launch_bounds__(64) void search_kernel(SearchArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int qi = blockIdx.x;
  if (qi >= a.nq) return;
  const int lane = lane_id();
  const int Lp = a.L_pow2;
  WaveCtx w;
  w.pool = reinterpret_cast<uint64_t*>(smem);
  w.next = w.pool + Lp;
  w.kept = w.next + Lp;
  w.cid = reinterpret_cast<int32_t*>(w.kept + kWave);
  int32_t* slot = w.cid + kWave;                 // tier slots of the survivors
  void* vis_mem = reinterpret_cast<void*>(slot + kWave);
  // With a tier the FP32 store sits in host memory (segments a.hsegs) behind
  // an HBM cache.  An FP32 traversal reads through the cache; a
  // reduced-precision traversal store stays in HBM and only the exact
  // re-scoring reads go through it.
  constexpr bool tier = TIER && sizeof(VT) == 4;
  // the traversal's gather: branch-free rounds for unscaled rows in HBM,
  // without any per-lane test when the rows fill their chunks (FULL)
  constexpr int form = (tier || Elem<VT>::kScaled) ? 0 : FULL ? 2 : 1;
  unsigned long long t_hit = 0, t_miss = 0;
  w.L = a.L;
  w.ktrack = a.last_change ? (a.k > 0 ? a.k : 1) : 0;
  VIS vis;
  vis.setup(vis_mem, a.T, a.id_bits);

  for (int i = lane; i < 2 * Lp; i += kWave) w.pool[i] = kKeyInf;

  using QS = QuerySlice<VT, NC>;
  QS qs;
  const int64_t qrow = a.qids ? (int64_t)a.qids[qi] : (int64_t)qi;
  qs.load(a.queries + qrow * a.qstride, a.dim, lane % QS::kLanesPerVec);
  const VT* base = reinterpret_cast<const VT*>(a.vec);
  __syncthreads();

  int n_dist = 0, n_exp = 0;

  // ---- InitCandidatePool ------------------------------------------------------
  // Random entries: the first min(E, n_alive) distinct alive ids in the order
  // of the query's own SplitMix64 stream.  Listed entries (learned form): every
  // distinct alive id of the query's list; a list with no usable id falls back
  // to random entries.  In both cases the best L keys start the pool.  Accepted
  // ids sit in an exact list that borrows the visited-table LDS.
  {
    int32_t* acc = static_cast<int32_t*>(vis_mem);
    int got = 0;
    auto accept_chunk = [&](int32_t id, bool valid, int want) {
      bool dup = false;
      for (int t = 0; t < kWave; ++t) {
        const int32_t o = __shfl(id, t);
        dup |= (t < lane) && (o == id);
      }
      for (int i = 0; i < got; ++i) dup |= acc[i] == id;
      const bool cand = valid && !dup;
      const uint64_t cb = ballot(cand);
      const int r = lanes_below(cb);
      const int room = want - got;
      const bool take = cand && r < room;
      __syncthreads();
      if (take) {
        acc[got + r] = id;
        w.cid[r] = id;
        if (tier) slot[r] = a.tmap[id];
      }
      const int nt = popc64(cb) < room ? popc64(cb) : room;
      got += nt;
      __syncthreads();
      if (tier) {
        const bool h = lane < nt && slot[lane] >= 0;
        t_hit += popc64(ballot(h));
        t_miss += nt - popc64(ballot(h));
      }
      uint64_t k = gather_keys<VT, NC, tier, form>(qs, base, a.vstride, w.cid, nt, a.metric, slot,
                                             reinterpret_cast<const VT*>(a.tcache), a.vscale,
                                             a.hsegs);
      n_dist += nt;
      sort_merge(w, k);
    };
    const int list = a.q_entry ? a.q_entry[qi] : -1;
    if (list >= 0) {
      const int32_t* ent = a.entry_lists + (int64_t)list * a.entry_cap;
      const int want = a.entry_cap;
      for (int j0 = 0; j0 < a.entry_cap && got < want; j0 += kWave) {
        const int j = j0 + lane;
        const int32_t id = j < a.entry_cap ? ent[j] : -1;
        const bool valid = id >= 0 && id < a.n_slots && alive_bit(a.alive, id);
        accept_chunk(id, valid, want);
      }
    }
    if (got == 0) {
      const uint64_t skey = a.qkey[qi];
      const int E = a.E;
      const int want = E < a.n_alive ? E : a.n_alive;
      const int attempts = 8 * E + 64;
      for (int a0 = 0; a0 < attempts && got < want; a0 += kWave) {
        const int j = a0 + lane;
        int32_t id = -1;
        bool valid = false;
        if (j < attempts) {
          id = range_reduce(splitmix64_at(skey, (uint64_t)j), (uint32_t)a.n_slots);
          valid = alive_bit(a.alive, id);
        }
        accept_chunk(id, valid, want);
      }
    }
    __syncthreads();
    vis.clear(a.T);
    __syncthreads();
    for (int i = lane; i < a.L; i += kWave) {
      const int32_t id = key_id(w.pool[i]);
      if (id >= 0) (void)vis.test_and_set(id);
    }
    __syncthreads();
  }

  // ---- repeat: nearest unexpanded -> neighbours -> distances -> update ------
  // Each iteration expands the `width` smallest unexpanded entries (one by
  // default); their rows are filtered, gathered and merged chunk by chunk,
  // which equals one merge of all new keys (the top-L of a union).
  const int cap_iters = (a.q_max_iters && a.q_max_iters[qi] > 0) ? a.q_max_iters[qi] : a.max_iters;
  int last_change = 0, n_iter = 0;
  const bool any_deleted = a.n_alive < a.n_slots;
  // FP8 rows whose vector scales sit beside the ids (a.nscale): each
  // survivor's scale goes to LDS with its id (in the slot array, which an
  // untiered traversal does not use) and no per-vector scale is read
  const bool rowsc = Elem<VT>::kScaled && !tier && a.nscale != nullptr;
  float* cscale = reinterpret_cast<float*>(slot);
  for (;;) {
    if (cap_iters > 0 && n_iter >= cap_iters) break;
    int ppos[4];
    int np = 0;
    for (int b0 = 0; b0 < a.L && np < a.width; b0 += kWave) {
      const int i = b0 + lane;
      const bool un = i < a.L && (w.pool[i] & 1ull) == 0;
      uint64_t bm = ballot(un);
      while (bm && np < a.width) {
        ppos[np++] = b0 + __ffsll((unsigned long long)bm) - 1;
        bm &= bm - 1;
      }
    }
    if (np == 0) break;
    int32_t parents[4];
    for (int t = 0; t < np; ++t) parents[t] = key_id(w.pool[ppos[t]]);
    __syncthreads();
    if (lane == 0) {
      for (int t = 0; t < np; ++t) {
        w.pool[ppos[t]] |= 1ull;
        if (TIER && a.trace && n_exp + t < a.trace_cap)
          a.trace[(int64_t)qi * a.trace_cap + n_exp + t] = parents[t];
      }
    }
    n_exp += np;
    ++n_iter;
    for (int t = 0; t < np; ++t) {
      const int32_t* row = a.graph + (int64_t)parents[t] * a.R;
      const float* rsc = a.nscale + (int64_t)parents[t] * a.R;
      for (int r0 = 0; r0 < a.R; r0 += kWave) {
        const int rr = r0 + lane;
        const int32_t nb = rr < a.R ? row[rr] : -1;
        const float nsc = rowsc && rr < a.R ? rsc[rr] : 0.0f;
        bool ok = nb >= 0 && nb < a.n_slots;
        // Deleted vertices are never evaluated.  With deletions in the
        // snapshot their bits load while the visited table is probed; with
        // none, no bit is read.
        uint32_t aword = ~0u;
        if (ok && any_deleted) aword = a.alive[(uint32_t)nb >> 5];
        __syncthreads();
        if (ok) ok = !vis.test_and_set(nb);
        if (ok && any_deleted) ok = (aword >> (nb & 31)) & 1u;
        const uint64_t ob = ballot(ok);
        if (ok) {
          w.cid[lanes_below(ob)] = nb;
          if (tier) slot[lanes_below(ob)] = a.tmap[nb];
          else if (rowsc) cscale[lanes_below(ob)] = nsc;
        }
        const int m = popc64(ob);
        __syncthreads();
        if (m == 0) continue;
        if (tier) {
          const bool h = lane < m && slot[lane] >= 0;
          t_hit += popc64(ballot(h));
          t_miss += m - popc64(ballot(h));
        }
        const uint64_t k = gather_keys<VT, NC, tier, form>(qs, base, a.vstride, w.cid, m, a.metric,
                                                     slot, reinterpret_cast<const VT*>(a.tcache),
                                                     a.vscale, a.hsegs, rowsc ? cscale : nullptr);
        n_dist += m;
        if (sort_merge(w, k)) last_change = n_iter;
      }
    }
  }

  // ---- exact re-scoring of the final pool (reduced-precision traversal) ------
  // an FP32 traversal is exact already: only reduced-precision kernels carry
  // the re-score
  if constexpr (!std::is_same<VT, float>::value) if (a.rerank) {
    QuerySlice<float, NC> q32;
    q32.load(a.queries + qrow * a.qstride, a.dim, lane % QuerySlice<float, NC>::kLanesPerVec);
    uint64_t* buf = w.next;
    for (int c0 = 0; c0 < a.L; c0 += kWave) {
      const int i = c0 + lane;
      const uint64_t pk = i < a.L ? w.pool[i] : kKeyInf;
      const int32_t id = key_id(pk);
      const bool on = id >= 0;
      const uint64_t ob = ballot(on);
      if (on) {
        w.cid[lanes_below(ob)] = id;
        if (TIER) slot[lanes_below(ob)] = a.tmap[id];
      }
      const int m = popc64(ob);
      __syncthreads();
      if (TIER) {
        const bool h = lane < m && slot[lane] >= 0;
        t_hit += popc64(ballot(h));
        t_miss += m - popc64(ballot(h));
      }
      const uint64_t k = gather_keys<float, NC, TIER>(q32, a.vec32, a.stride, w.cid, m, a.metric,
                                                      slot, a.tcache, nullptr, a.hsegs);
      if (lane < m) buf[c0 + lane] = k;
      else if (c0 + lane < Lp) buf[c0 + lane] = kKeyInf;
      __syncthreads();
    }
    for (int i = a.L + lane; i < Lp; i += kWave) buf[i] = kKeyInf;
    __syncthreads();
    wave_sort_lds(buf, Lp < kWave ? kWave : Lp);
    uint64_t* t = w.pool; w.pool = w.next; w.next = t;
  }

  // ---- output -------------------------------------------------------------------
  if (a.out_pool) {
    for (int i = lane; i < a.L; i += kWave) {
      const uint64_t pk = w.pool[i];
      a.out_pool[(int64_t)qi * a.L + i] = pk == kKeyInf ? kKeyInf : (pk & ~1ull);
    }
  }
  if (a.out_ids) {
    for (int i = lane; i < a.k; i += kWave) {
      const uint64_t pk = w.pool[i];
      a.out_ids[(int64_t)qi * a.k + i] = key_id(pk);
      a.out_d[(int64_t)qi * a.k + i] = key_dist(pk);
    }
  }
  if (lane == 0) {
    if (a.n_dist) a.n_dist[qi] = n_dist;
    if (a.n_exp) a.n_exp[qi] = n_exp;
    if (a.last_change) a.last_change[qi] = last_change;
    if (TIER && a.trace_n) a.trace_n[qi] = n_exp;
    if (TIER && a.tier_counts) {
      atomicAdd(&a.tier_counts[0], t_hit);
      atomicAdd(&a.tier_counts[1], t_miss);
    }
    if (a.totals) {
      atomicAdd(&a.totals[0], (unsigned long long)n_dist);
      atomicAdd(&a.totals[1], (unsigned long long)n_exp);
    }
  }
}

// Per-query stream key: seed XOR FNV-1a 64 over the query's FP32 bytes
// (little-endian, element order).  One thread per query.
__global__ void query_key_kernel(const float* __restrict__ q, int64_t qstride, const int32_t* qids,
                                 int dim, int nq, uint64_t seed, uint64_t* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  const int64_t row = qids ? (int64_t)qids[i] : (int64_t)i;
  const uint32_t* w = reinterpret_cast<const uint32_t*>(q + row * qstride);
  uint64_t h = kFnvBasis;
  for (int t = 0; t < dim; ++t) {
    const uint32_t x = w[t];
#pragma unroll
    for (int b = 0; b < 4; ++b) { h ^= (x >> (8 * b)) & 0xffu; h *= kFnvPrime; }
  }
  out[i] = seed ^ h;
}

// ---------------------------------------------------------------------------
// Visited-table layout: T / 4 sets of packed tags (T * 2 bytes) when the ids
// fit (tag width id_bits - log2(sets) <= 15), else T 32-bit ids.
static int id_bits_for(int32_t n_slots) {
  int b = 1;
  while (b < 31 && (1ll << b) < (long long)n_slots) ++b;
  return b;
}
static bool use_tags(int32_t n_slots, int T) {
  int set_bits = 0;
  while ((1 << (set_bits + 1)) <= T / 4) ++set_bits;
  int b = id_bits_for(n_slots);
  if (b < set_bits + 1) b = set_bits + 1;
  return b - set_bits <= 15;
}
static size_t vis_bytes(int T, bool tags) { return tags ? (size_t)T * 2 : (size_t)T * 4; }

template <typename VT, typename VIS, bool TIER, bool FULL>
static hipError_t launch_nc(const SearchArgs& a, int nc, size_t lds, hipStream_t st) {
  dim3 grid(a.nq), block(kWave);
  switch (nc) {
    case 1: hipLaunchKernelGGL((search_kernel<VT, 1, VIS, TIER, FULL>), grid, block, lds, st, a); break;
    case 2: hipLaunchKernelGGL((search_kernel<VT, 2, VIS, TIER, FULL>), grid, block, lds, st, a); break;
    case 4: hipLaunchKernelGGL((search_kernel<VT, 4, VIS, TIER, FULL>), grid, block, lds, st, a); break;
    case 8: hipLaunchKernelGGL((search_kernel<VT, 8, VIS, TIER, FULL>), grid, block, lds, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Rows that fill all nc chunks of 128 elements (stride 128, 256, 512, 1024)
// take the kernel whose gather loads carry no per-lane test.  Kernels that
// gather with the predicated form either way have no such twin.
template <typename VT, typename VIS, bool TIER>
static hipError_t launch_vt(const SearchArgs& a, int nc, size_t lds, hipStream_t st) {
  constexpr bool kTwin = !Elem<VT>::kScaled && !(TIER && sizeof(VT) == 4);
  if constexpr (kTwin)
    if (a.vstride >= (int64_t)nc * 128) return launch_nc<VT, VIS, TIER, true>(a, nc, lds, st);
  return launch_nc<VT, VIS, TIER, false>(a, nc, lds, st);
}

template <typename VIS>
static hipError_t launch_vis(const SearchArgs& a, int precision, int nc, size_t lds, hipStream_t st) {
  switch (precision) {
    case 0:
      return a.tmap ? launch_vt<float, VIS, true>(a, nc, lds, st)
                    : launch_vt<float, VIS, false>(a, nc, lds, st);
    case 1:
      return a.tmap ? launch_vt<__half, VIS, true>(a, nc, lds, st)
                    : launch_vt<__half, VIS, false>(a, nc, lds, st);
    case 2:
      return a.tmap ? launch_vt<bf16_t, VIS, true>(a, nc, lds, st)
                    : launch_vt<bf16_t, VIS, false>(a, nc, lds, st);
    case 3:
      if (!a.vscale || a.vstride % 16) return hipErrorInvalidValue;
      return a.tmap ? launch_vt<fp8_t, VIS, true>(a, nc, lds, st)
                    : launch_vt<fp8_t, VIS, false>(a, nc, lds, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_search(const SearchArgs& in, int precision, hipStream_t st) {
  if (in.nq <= 0) return hipSuccess;
  SearchArgs a = in;
  if (a.vstride == 0) a.vstride = a.stride;
  const int chunks = (int)((a.stride + 127) / 128);
  const int nc = chunks <= 1 ? 1 : chunks <= 2 ? 2 : chunks <= 4 ? 4 : 8;
  if (chunks > 8) return hipErrorInvalidValue;
  const bool assoc = a.vis_compact && use_tags(a.n_slots, a.T);
  // the entry phase keeps its exact list of accepted ids in the table's LDS
  while (vis_bytes(a.T, assoc) < (size_t)a.E * 4) a.T <<= 1;
  int set_bits = 0;
  while ((1 << (set_bits + 1)) <= a.T / 4) ++set_bits;
  a.id_bits = id_bits_for(a.n_slots);
  if (a.id_bits < set_bits + 1) a.id_bits = set_bits + 1;
  int Lp = 64;
  while (Lp < a.L) Lp <<= 1;
  a.L_pow2 = Lp;
  if (coop_eligible(a, precision, nc))
    return launch_search_coop(a, precision, nc, assoc, vis_bytes(a.T, assoc), st);
  const size_t lds = (size_t)2 * Lp * 8 + kWave * 8 + 2 * kWave * 4 + vis_bytes(a.T, assoc);
  return assoc ? launch_vis<VisTags>(a, precision, nc, lds, st)
               : launch_vis<VisLinear32>(a, precision, nc, lds, st);
}

hipError_t launch_query_keys(const float* q, int64_t qstride, const int32_t* qids, int dim, int nq,
                             uint64_t seed, uint64_t* out, hipStream_t st) {
  if (nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(query_key_kernel, dim3((nq + 255) / 256), dim3(256), 0, st, q, qstride, qids,
                     dim, nq, seed, out);
  return hipGetLastError();
}

}  // namespace svf
