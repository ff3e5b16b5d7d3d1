// Best-first search with W waves per query (Algorithm 1 with W parents per
// iteration): for small batches, where one wave per query would leave most
// of the chip idle, the waves of one workgroup share the query's pool and
// visited table and each expands one of the W smallest unexpanded entries of
// an iteration.  The result is that of the W-parent search of the one-wave
// kernel: the pool after an iteration is the top L of the old pool and all
// new keys, with equal keys kept once.
//
// Per iteration every wave finds the same W parents; after a barrier each
// wave marks its parent, filters the parent's row through the shared visited
// table (a race between waves can only make an id be evaluated twice, and
// the two equal keys collapse in the merge), gathers the survivors, drops
// keys that cannot enter the pool or that the pool already holds, and sorts
// the rest.  After a barrier each wave drops keys that an earlier wave also
// produced; after another, all threads place every surviving key at its
// rank (the count of smaller keys over the pool and the W lists) in the next
// pool.  The entry phase, the exact re-scoring and the output run on wave 0.
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"
#include "wave_ops.hpp"

namespace svf {

namespace {

// Keys of a sorted list (by key_ord) below k.
__device__ __forceinline__ int count_below(const uint64_t* a, int n, uint64_t k) {
  const uint64_t o = key_ord(k);
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (key_ord(a[mid]) < o) lo = mid + 1; else hi = mid;
  }
  return lo;
}
__device__ __forceinline__ bool holds(const uint64_t* a, int n, uint64_t k) {
  const int i = count_below(a, n, k);
  return i < n && key_ord(a[i]) == key_ord(k);
}

}  // namespace

template <typename VT, int NC, typename VIS, int W>
__global__ __launch_bounds__(64 * W) void search_coop_kernel(SearchArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int qi = blockIdx.x;
  if (qi >= a.nq) return;
  const int wv = threadIdx.x / kWave, lane = lane_id();
  const int Lp = a.L_pow2, L = a.L;
  uint64_t* bufA = reinterpret_cast<uint64_t*>(smem);
  uint64_t* bufB = bufA + Lp;
  uint64_t* lst = bufB + Lp;                                   // W x 64 sorted new keys
  uint64_t* kept = lst + W * kWave;                            // W x 64 staging
  int32_t* cid = reinterpret_cast<int32_t*>(kept + W * kWave); // W x 64 survivor ids
  int32_t* meta = cid + W * kWave;                             // 64 ints
  void* vis_mem = reinterpret_cast<void*>(meta + kWave);
  VIS vis;
  vis.setup(vis_mem, a.T, a.id_bits);
  for (int i = threadIdx.x; i < 2 * Lp; i += kWave * W) bufA[i] = kKeyInf;

  using QS = QuerySlice<VT, NC>;
  QS qs;
  const int64_t qrow = a.qids ? (int64_t)a.qids[qi] : (int64_t)qi;
  qs.load(a.queries + qrow * a.qstride, a.dim, lane % QS::kLanesPerVec);
  const VT* base = reinterpret_cast<const VT*>(a.vec);
  int32_t* mycid = cid + wv * kWave;
  const int ktrack = a.last_change ? (a.k > 0 ? a.k : 1) : 0;
  int n_dist = 0;
  __syncthreads();

  // ---- entry phase on wave 0 (as in the one-wave kernel) ----------------------
  if (wv == 0) {
    WaveCtx w;
    w.pool = bufA;
    w.next = bufB;
    w.kept = kept;
    w.cid = cid;
    w.L = L;
    w.ktrack = 0;
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
      WaveSync::sync();
      if (take) {
        acc[got + r] = id;
        cid[r] = id;
      }
      const int nt = popc64(cb) < room ? popc64(cb) : room;
      got += nt;
      WaveSync::sync();
      uint64_t k = gather_keys<VT, NC, false>(qs, base, a.vstride, cid, nt, a.metric, nullptr,
                                              nullptr, a.vscale);
      n_dist += nt;
      sort_merge<WaveSync>(w, k);
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
    WaveSync::sync();
    if (w.pool != bufA)
      for (int i = lane; i < Lp; i += kWave) bufA[i] = w.pool[i];
    WaveSync::sync();
    vis.clear(a.T);
    WaveSync::sync();
    for (int i = lane; i < L; i += kWave) {
      const int32_t id = key_id(bufA[i]);
      if (id >= 0) (void)vis.test_and_set(id);
    }
    if (lane == 0) {
      int valid = 0;
      while (valid < L && bufA[valid] != kKeyInf) ++valid;
      meta[2 * W + 1] = valid;
    }
  }
  __syncthreads();

  // ---- W parents per iteration ------------------------------------------------
  uint64_t* cur = bufA;
  uint64_t* nxt = bufB;
  int lcur = meta[2 * W + 1];
  const int cap_iters = (a.q_max_iters && a.q_max_iters[qi] > 0) ? a.q_max_iters[qi] : a.max_iters;
  int last_change = 0, n_iter = 0, n_exp = 0;
  const bool any_deleted = a.n_alive < a.n_slots;
  for (;;) {
    if (cap_iters > 0 && n_iter >= cap_iters) break;
    int ppos[W];
    int np = 0;
    for (int b0 = 0; b0 < L && np < W; b0 += kWave) {
      const int i = b0 + lane;
      const bool un = i < L && (cur[i] & 1ull) == 0;
      uint64_t bm = ballot(un);
      while (bm && np < W) {
        ppos[np++] = b0 + __ffsll((unsigned long long)bm) - 1;
        bm &= bm - 1;
      }
    }
    if (np == 0) break;
    const bool active = wv < np;
    int32_t parent = -1;
    for (int t = 0; t < W; ++t)
      if (t == wv && active) parent = key_id(cur[ppos[t]]);
    const uint64_t last = cur[L - 1];
    __syncthreads();
    if (active && lane == 0) {
      for (int t = 0; t < W; ++t)
        if (t == wv) cur[ppos[t]] |= 1ull;
    }
    n_exp += np;
    ++n_iter;
    int mw = 0;
    if (active) {
      const int32_t nb = lane < a.R ? a.graph[(int64_t)parent * a.R + lane] : -1;
      bool ok = nb >= 0 && nb < a.n_slots;
      // deleted vertices are never evaluated (no bit is read without deletions)
      uint32_t aword = ~0u;
      if (ok && any_deleted) aword = a.alive[(uint32_t)nb >> 5];
      if (ok) ok = !vis.test_and_set(nb);
      if (ok && any_deleted) ok = (aword >> (nb & 31)) & 1u;
      const uint64_t ob = ballot(ok);
      if (ok) mycid[lanes_below(ob)] = nb;
      const int m = popc64(ob);
      WaveSync::sync();
      uint64_t k = kKeyInf;
      if (m > 0) {
        k = gather_keys<VT, NC, false>(qs, base, a.vstride, mycid, m, a.metric, nullptr, nullptr,
                                       a.vscale);
        n_dist += m;
      }
      // keys that can enter a full pool, sorted; then those the pool lacks
      const bool live = k != kKeyInf && (last == kKeyInf || key_ord(k) < key_ord(last));
      const uint64_t lb = ballot(live);
      const int s = popc64(lb);
      uint64_t* mykept = kept + wv * kWave;
      if (live) mykept[lanes_below(lb)] = k;
      WaveSync::sync();
      uint64_t c = lane < s ? mykept[lane] : kKeyInf;
      int Wd = 1;
      while (Wd < s) Wd <<= 1;
      c = wave_sort_width(c, Wd);
      const bool keep = c != kKeyInf && !holds(cur, lcur, c);
      const uint64_t kb = ballot(keep);
      uint64_t* mylst = lst + wv * kWave;
      if (keep) mylst[lanes_below(kb)] = c;
      mw = popc64(kb);
    }
    if (lane == 0) meta[wv] = mw;
    __syncthreads();
    // keys an earlier wave also produced are dropped (order kept); the lists
    // are only read here, the survivors go to the staging rows
    {
      const uint64_t* mylst = lst + wv * kWave;
      const uint64_t e = lane < mw ? mylst[lane] : kKeyInf;
      bool dup = false;
      for (int v = 0; v < W; ++v)
        if (v < wv && lane < mw) dup |= holds(lst + v * kWave, meta[v], e);
      const bool keep = lane < mw && !dup;
      const uint64_t kb = ballot(keep);
      if (keep) kept[wv * kWave + lanes_below(kb)] = e;
      if (lane == 0) meta[W + wv] = popc64(kb);
    }
    __syncthreads();
    const uint64_t* fin = kept;   // W x 64 sorted, distinct new keys
    int cnt[W];
    int total = lcur;
    for (int v = 0; v < W; ++v) {
      cnt[v] = meta[W + v];
      total += cnt[v];
    }
    const int lnext = total < L ? total : L;
    int changed = 0;
    for (int idx = threadIdx.x; idx < total; idx += kWave * W) {
      uint64_t e;
      int rank;
      bool fresh = false;
      if (idx < lcur) {
        e = cur[idx];
        rank = idx;
        for (int v = 0; v < W; ++v) rank += count_below(fin + v * kWave, cnt[v], e);
      } else {
        int j = idx - lcur, src = 0;
        for (int v = 0; v < W; ++v)
          if (j >= cnt[v] && v == src) { j -= cnt[v]; ++src; }
        e = fin[src * kWave + j];
        fresh = true;
        rank = count_below(cur, lcur, e) + j;
        for (int v = 0; v < W; ++v)
          if (v != src) rank += count_below(fin + v * kWave, cnt[v], e);
      }
      if (rank < L) nxt[rank] = e;
      if (fresh && rank < ktrack) changed = 1;
    }
    for (int i = lnext + (int)threadIdx.x; i < L; i += kWave * W) nxt[i] = kKeyInf;
    if (ktrack > 0) {
      if (threadIdx.x == 0) meta[2 * W] = 0;
      __syncthreads();
      if (changed) meta[2 * W] = 1;
    }
    __syncthreads();
    if (ktrack > 0 && meta[2 * W]) last_change = n_iter;
    uint64_t* t = cur; cur = nxt; nxt = t;
    lcur = lnext;
  }
  if (lane == 0) meta[wv] = n_dist;
  __syncthreads();

  // ---- exact re-scoring, output (wave 0) -----------------------------------------
  if (wv != 0) return;
  int nd_all = 0;
  for (int v = 0; v < W; ++v) nd_all += meta[v];
  // an FP32 traversal is exact already: only reduced-precision kernels carry
  // the re-score
  if constexpr (!std::is_same<VT, float>::value) if (a.rerank) {
    QuerySlice<float, NC> q32;
    q32.load(a.queries + qrow * a.qstride, a.dim, lane % QuerySlice<float, NC>::kLanesPerVec);
    uint64_t* buf = nxt;
    for (int c0 = 0; c0 < L; c0 += kWave) {
      const int i = c0 + lane;
      const uint64_t pk = i < L ? cur[i] : kKeyInf;
      const int32_t id = key_id(pk);
      const bool on = id >= 0;
      const uint64_t ob = ballot(on);
      if (on) cid[lanes_below(ob)] = id;
      const int m = popc64(ob);
      WaveSync::sync();
      const uint64_t k = gather_keys<float, NC>(q32, a.vec32, a.stride, cid, m, a.metric);
      if (lane < m) buf[c0 + lane] = k;
      else if (c0 + lane < Lp) buf[c0 + lane] = kKeyInf;
      WaveSync::sync();
    }
    for (int i = L + lane; i < Lp; i += kWave) buf[i] = kKeyInf;
    WaveSync::sync();
    wave_sort_lds<WaveSync>(buf, Lp < kWave ? kWave : Lp);
    cur = buf;
  }
  if (a.out_pool) {
    for (int i = lane; i < L; i += kWave) {
      const uint64_t pk = cur[i];
      a.out_pool[(int64_t)qi * L + i] = pk == kKeyInf ? kKeyInf : (pk & ~1ull);
    }
  }
  if (a.out_ids) {
    for (int i = lane; i < a.k; i += kWave) {
      const uint64_t pk = cur[i];
      a.out_ids[(int64_t)qi * a.k + i] = key_id(pk);
      a.out_d[(int64_t)qi * a.k + i] = key_dist(pk);
    }
  }
  if (lane == 0) {
    if (a.n_dist) a.n_dist[qi] = nd_all;
    if (a.n_exp) a.n_exp[qi] = n_exp;
    if (a.last_change) a.last_change[qi] = last_change;
    if (a.totals) {
      atomicAdd(&a.totals[0], (unsigned long long)nd_all);
      atomicAdd(&a.totals[1], (unsigned long long)n_exp);
    }
  }
}

template <typename VT, typename VIS, int W>
static hipError_t launch_coop_w(const SearchArgs& a, int nc, size_t lds, hipStream_t st) {
  dim3 grid(a.nq), block(kWave * W);
  switch (nc) {
    case 1: hipLaunchKernelGGL((search_coop_kernel<VT, 1, VIS, W>), grid, block, lds, st, a); break;
    case 2: hipLaunchKernelGGL((search_coop_kernel<VT, 2, VIS, W>), grid, block, lds, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename VIS>
static hipError_t launch_coop_vis(const SearchArgs& a, int precision, int nc, size_t lds,
                                  hipStream_t st) {
  const bool w4 = a.width == 4;
  switch (precision) {
    case 0: return w4 ? launch_coop_w<float, VIS, 4>(a, nc, lds, st)
                      : launch_coop_w<float, VIS, 2>(a, nc, lds, st);
    case 2: return w4 ? launch_coop_w<bf16_t, VIS, 4>(a, nc, lds, st)
                      : launch_coop_w<bf16_t, VIS, 2>(a, nc, lds, st);
    case 3: return w4 ? launch_coop_w<fp8_t, VIS, 4>(a, nc, lds, st)
                      : launch_coop_w<fp8_t, VIS, 2>(a, nc, lds, st);
  }
  return hipErrorInvalidValue;
}

bool coop_eligible(const SearchArgs& a, int precision, int nc) {
  return a.coop_max_nq > 0 && a.nq <= a.coop_max_nq && (a.width == 2 || a.width == 4) &&
         a.R <= kWave && nc <= 2 && !a.tmap && precision != 1;
}

hipError_t launch_search_coop(const SearchArgs& a, int precision, int nc, bool tags, size_t vis,
                              hipStream_t st) {
  const int W = a.width;
  const size_t lds = (size_t)2 * a.L_pow2 * 8 + (size_t)W * kWave * (8 + 8 + 4) + kWave * 4 + vis;
  return tags ? launch_coop_vis<VisTags>(a, precision, nc, lds, st)
              : launch_coop_vis<VisLinear32>(a, precision, nc, lds, st);
}

}  // namespace svf
