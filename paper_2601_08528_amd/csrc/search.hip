// Batched best-first graph search (SVFusion, Sec. 4.2, Algorithm 1) on one
// device tier, one wavefront per query.
//
// Per query the wave keeps in LDS
//   - the candidate pool: `L` sorted 64-bit keys (dist, id, expanded flag),
//     double-buffered so a merge writes the next pool while reading this one;
//   - a visited table of T id slots (open addressing).  During the entry phase
//     it is exact; afterwards a probe sequence of kProbe slots that finds
//     neither the id nor a free slot overwrites its first slot, so the table
//     may forget ids but never reports an unvisited id as visited.  Forgetting
//     costs only repeated distance evaluations: an id that left the pool had
//     L smaller keys, the L-th key never grows, so it is rejected again, and an
//     id still in the pool is recognised by its identical key during the merge.
//
// One iteration: the smallest unexpanded key is the parent (Algorithm 1,
// GetNearest); its row of R ids is read with one coalesced load; ids that are
// INVALID, deleted (bitset) or visited are dropped; the survivors are compacted
// and their vectors gathered so that each 16-lane (16-bit store) or 32-lane
// (FP32 store) group reads one 256/512-byte vector with 16-byte loads; the
// group reduces its partial sums by lane shuffles; the new keys are sorted
// across the wave (bitonic) and merged into the pool by rank (merge path),
// which also drops re-evaluated ids.  The loop ends when every pool entry is
// expanded (or after max_iters expansions).
#include "common.hpp"
#include "kernels.hpp"
#include "wave_ops.hpp"

namespace svf {


// ---------------------------------------------------------------------------
template <typename VT, int NC>
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
  w.vis = reinterpret_cast<uint32_t*>(w.cid + kWave);
  w.tmask = (uint32_t)a.T - 1u;
  w.L = a.L;

  for (int i = lane; i < a.T; i += kWave) w.vis[i] = kEmpty;
  for (int i = lane; i < 2 * Lp; i += kWave) w.pool[i] = kKeyInf;

  using QS = QuerySlice<VT, NC>;
  QS qs;
  const int64_t qrow = a.qids ? (int64_t)a.qids[qi] : (int64_t)qi;
  qs.load(a.queries + qrow * a.qstride, a.dim, lane % QS::kLanesPerVec);
  const VT* base = reinterpret_cast<const VT*>(a.vec);
  __syncthreads();

  int n_dist = 0, n_exp = 0;

  // ---- InitCandidatePool: random entries from the query's own stream -------
  const uint64_t skey = a.qkey[qi];
  const int E = a.E;
  const int want = E < a.n_alive ? E : a.n_alive;
  const int attempts = 8 * E + 64;
  int got = 0;
  for (int a0 = 0; a0 < attempts && got < want; a0 += kWave) {
    const int j = a0 + lane;
    int32_t id = -1;
    bool valid = false;
    if (j < attempts) {
      id = range_reduce(splitmix64_at(skey, (uint64_t)j), (uint32_t)a.n_slots);
      valid = alive_bit(a.alive, id);
    }
    bool dup = false;
    for (int t = 0; t < kWave; ++t) {
      const int32_t o = __shfl(id, t);
      dup |= (t < lane) && (o == id);
    }
    const bool cand = valid && !dup && !vis_contains_exact(w.vis, w.tmask, id);
    const uint64_t cb = ballot(cand);
    const int r = lanes_below(cb);
    const int room = want - got;
    const bool take = cand && r < room;
    __syncthreads();
    if (take) { vis_insert_exact(w.vis, w.tmask, id); w.cid[r] = id; }
    const int nt = popc64(cb) < room ? popc64(cb) : room;
    got += nt;
    __syncthreads();
    uint64_t k = gather_keys<VT, NC>(qs, base, a.stride, w.cid, nt, a.metric);
    n_dist += nt;
    k = wave_sort64(k);
    merge_into_pool(w, k);
  }

  // ---- repeat: nearest unexpanded -> neighbours -> distances -> update ------
  for (;;) {
    if (a.max_iters > 0 && n_exp >= a.max_iters) break;
    int ppos = -1;
    for (int b0 = 0; b0 < a.L; b0 += kWave) {
      const int i = b0 + lane;
      const bool un = i < a.L && (w.pool[i] & 1ull) == 0;
      const uint64_t bm = ballot(un);
      if (bm) { ppos = b0 + __ffsll((unsigned long long)bm) - 1; break; }
    }
    if (ppos < 0) break;
    const uint64_t pk = w.pool[ppos];
    const int32_t parent = key_id(pk);
    __syncthreads();
    if (lane == 0) w.pool[ppos] = pk | 1ull;
    ++n_exp;
    const int32_t* row = a.graph + (int64_t)parent * a.R;
    for (int r0 = 0; r0 < a.R; r0 += kWave) {
      const int rr = r0 + lane;
      int32_t nb = rr < a.R ? row[rr] : -1;
      bool ok = nb >= 0 && nb < a.n_slots && alive_bit(a.alive, nb);
      __syncthreads();
      if (ok) ok = !vis_test_and_set(w.vis, w.tmask, nb);
      const uint64_t ob = ballot(ok);
      if (ok) w.cid[lanes_below(ob)] = nb;
      const int m = popc64(ob);
      __syncthreads();
      if (m == 0) continue;
      uint64_t k = gather_keys<VT, NC>(qs, base, a.stride, w.cid, m, a.metric);
      n_dist += m;
      k = wave_sort64(k);
      merge_into_pool(w, k);
    }
  }

  // ---- exact re-scoring of the final pool (reduced-precision traversal) ------
  if (a.rerank) {
    QuerySlice<float, NC> q32;
    q32.load(a.queries + qrow * a.qstride, a.dim, lane % QuerySlice<float, NC>::kLanesPerVec);
    uint64_t* buf = w.next;
    for (int c0 = 0; c0 < a.L; c0 += kWave) {
      const int i = c0 + lane;
      const uint64_t pk = i < a.L ? w.pool[i] : kKeyInf;
      const int32_t id = key_id(pk);
      const bool on = id >= 0;
      const uint64_t ob = ballot(on);
      if (on) w.cid[lanes_below(ob)] = id;
      const int m = popc64(ob);
      __syncthreads();
      const uint64_t k = gather_keys<float, NC>(q32, a.vec32, a.stride, w.cid, m, a.metric);
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
size_t search_lds_bytes(int L, int T) {
  int Lp = 64;
  while (Lp < L) Lp <<= 1;
  return (size_t)2 * Lp * 8 + kWave * 8 + kWave * 4 + (size_t)T * 4;
}

template <typename VT>
static hipError_t launch_vt(const SearchArgs& a, int nc, hipStream_t st) {
  const size_t lds = search_lds_bytes(a.L, a.T);
  dim3 grid(a.nq), block(kWave);
  switch (nc) {
    case 1: hipLaunchKernelGGL((search_kernel<VT, 1>), grid, block, lds, st, a); break;
    case 2: hipLaunchKernelGGL((search_kernel<VT, 2>), grid, block, lds, st, a); break;
    case 4: hipLaunchKernelGGL((search_kernel<VT, 4>), grid, block, lds, st, a); break;
    case 8: hipLaunchKernelGGL((search_kernel<VT, 8>), grid, block, lds, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_search(const SearchArgs& a, int precision, hipStream_t st) {
  if (a.nq <= 0) return hipSuccess;
  const int chunks = (int)((a.stride + 127) / 128);
  const int nc = chunks <= 1 ? 1 : chunks <= 2 ? 2 : chunks <= 4 ? 4 : 8;
  if (chunks > 8) return hipErrorInvalidValue;
  switch (precision) {
    case 0: return launch_vt<float>(a, nc, st);
    case 1: return launch_vt<__half>(a, nc, st);
    case 2: return launch_vt<bf16_t>(a, nc, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_query_keys(const float* q, int64_t qstride, const int32_t* qids, int dim, int nq,
                             uint64_t seed, uint64_t* out, hipStream_t st) {
  if (nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(query_key_kernel, dim3((nq + 255) / 256), dim3(256), 0, st, q, qstride, qids,
                     dim, nq, seed, out);
  return hipGetLastError();
}

}  // namespace svf
