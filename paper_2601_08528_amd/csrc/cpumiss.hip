// Search with CPU-GPU co-processing of a tiered store (Sec. 4.2, Alg. 1):
// the neighbours of an expanded vertex are split by the cache's mapping table
// into X_GPU (cached rows, distances on the GPU) and X_CPU (uncached rows,
// distances on the host cores, where those rows live), and the two sets of
// distances update the candidate pool together.
//
// The batch advances in rounds.  A round kernel (one wave per query) takes
// each active query one step: the entry phase in round 0, else the nearest
// unexpanded pool entry is expanded and its unseen alive neighbours are
// split; cached ones are gathered from HBM at once, the others go to a miss
// list.  The host computes the listed distances on its cores, with the same
// FP32 operations in the same order as the GPU's gather (per-lane fused
// multiply-adds over 4-element slices, then an exchange tree over 32 lanes),
// so every distance equals the one the GPU would compute; a merge kernel then
// merges each query's new keys into its pool.  A query is done when no
// unexpanded entry is left (or at max_iters).  The pools live in HBM between
// rounds, and an id already in the pool is not evaluated again; ids evicted
// earlier may be, which changes no result (the L-th key never grows).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "common.hpp"
#include "index.hpp"
#include "index_internal.hpp"
#include "kernels.hpp"
#include "wave_ops.hpp"

namespace svf {

struct CoArgs {
  SearchArgs s;
  uint64_t* pool;      // nq x Lp pool keys (bit 0: expanded)
  int32_t* state;      // nq: 0 active, 1 done
  int32_t* iters;      // nq: expansions so far
  int32_t* ndist;      // nq
  uint64_t* newk;      // nq x C keys of the round (a miss holds a placeholder)
  int32_t* newn;       // nq
  int C;
  int32_t* miss_pos;   // index into newk of each listed miss
  int32_t* miss_id;
  int32_t* counters;   // [0] misses listed, [1] queries active this round
};

namespace {

template <int NC>
__global__ __launch_bounds__(64) void co_round_kernel(CoArgs c, int round) {
  extern __shared__ __align__(16) unsigned char smem[];
  const SearchArgs& a = c.s;
  const int qi = blockIdx.x;
  const int lane = lane_id();
  if (c.state[qi]) {
    if (lane == 0) c.newn[qi] = 0;
    return;
  }
  const int Lp = a.L_pow2;
  uint64_t* pool = reinterpret_cast<uint64_t*>(smem);
  int32_t* cid = reinterpret_cast<int32_t*>(pool + Lp);
  int32_t* slot = cid + kWave;
  uint32_t* tab = reinterpret_cast<uint32_t*>(slot + kWave);
  QuerySlice<float, NC> qs;
  const int64_t qrow = a.qids ? (int64_t)a.qids[qi] : (int64_t)qi;
  qs.load(a.queries + qrow * a.qstride, a.dim, lane % QuerySlice<float, NC>::kLanesPerVec);
  const float* host = reinterpret_cast<const float*>(a.vec);
  uint64_t* out = c.newk + (int64_t)qi * c.C;
  int n = 0;
  unsigned long long hits = 0, misses = 0;
  // the m ids in cid[]: cached ones gathered here, the others listed for the host
  auto split = [&](int m) {
    const bool on = lane < m;
    const int32_t id = on ? cid[lane] : -1;
    const int32_t sl = on ? a.tmap[id] : -1;
    const bool hit = on && sl >= 0;
    const bool miss = on && sl < 0;
    const uint64_t hb = ballot(hit), mb = ballot(miss);
    const int nh = popc64(hb), nm = popc64(mb);
    int mpos = 0;
    if (lane == 0 && nm > 0) mpos = atomicAdd(&c.counters[0], nm);
    mpos = __shfl(mpos, 0);
    if (miss) {
      const int r = lanes_below(mb);
      c.miss_pos[mpos + r] = (int32_t)((int64_t)qi * c.C + n + nh + r);
      c.miss_id[mpos + r] = id;
      out[n + nh + r] = kKeyInf;
    }
    __syncthreads();
    if (hit) {
      const int r = lanes_below(hb);
      cid[r] = id;
      slot[r] = sl;
    }
    __syncthreads();
    const uint64_t k = gather_keys<float, NC, true, 0>(qs, host, a.stride, cid, nh, a.metric, slot,
                                                      a.tcache, nullptr, a.hsegs);
    if (lane < nh) out[n + lane] = k;
    n += nh + nm;
    hits += nh;
    misses += nm;
    __syncthreads();
  };

  bool active = true;
  if (round == 0) {
    // InitCandidatePool: the first min(E, n_alive) distinct alive ids of the
    // query's SplitMix64 stream (the same ids as the one-kernel search)
    int32_t* acc = reinterpret_cast<int32_t*>(tab);
    int got = 0;
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
        cid[r] = id;
      }
      const int nt = popc64(cb) < room ? popc64(cb) : room;
      got += nt;
      __syncthreads();
      split(nt);
    }
  } else {
    const int cap = a.max_iters;
    if (cap > 0 && c.iters[qi] >= cap) {
      active = false;
    } else {
      uint64_t* gp = c.pool + (int64_t)qi * Lp;
      for (int i = lane; i < Lp; i += kWave) pool[i] = gp[i];
      // ids in the pool, for the filter
      const int S = 2 * Lp;
      const uint32_t mask = (uint32_t)S - 1u;
      for (int i = lane; i < S; i += kWave) tab[i] = kEmpty;
      __syncthreads();
      for (int i = lane; i < a.L; i += kWave)
        if (pool[i] != kKeyInf) vis_insert_exact(tab, mask, key_id(pool[i]));
      __syncthreads();
      int p = -1;
      for (int b0 = 0; b0 < a.L && p < 0; b0 += kWave) {
        const int i = b0 + lane;
        const bool un = i < a.L && pool[i] != kKeyInf && (pool[i] & 1ull) == 0;
        const uint64_t bm = ballot(un);
        if (bm) p = b0 + __ffsll((unsigned long long)bm) - 1;
      }
      if (p < 0) {
        active = false;
      } else {
        const int32_t parent = key_id(pool[p]);
        const int ne = c.iters[qi];
        if (lane == 0) {
          gp[p] = pool[p] | 1ull;
          c.iters[qi] = ne + 1;
          if (a.trace && ne < a.trace_cap) a.trace[(int64_t)qi * a.trace_cap + ne] = parent;
        }
        const int32_t* row = a.graph + (int64_t)parent * a.R;
        for (int r0 = 0; r0 < a.R; r0 += kWave) {
          const int rr = r0 + lane;
          const int32_t nb = rr < a.R ? row[rr] : -1;
          const bool ok = nb >= 0 && nb < a.n_slots && alive_bit(a.alive, nb) &&
                          !vis_contains_exact(tab, mask, nb);
          const uint64_t ob = ballot(ok);
          __syncthreads();
          if (ok) cid[lanes_below(ob)] = nb;
          __syncthreads();
          split(popc64(ob));
        }
      }
    }
  }
  if (lane == 0) {
    c.newn[qi] = n;
    c.ndist[qi] += n;
    if (!active) c.state[qi] = 1;
    else atomicAdd(&c.counters[1], 1);
    if (a.tier_counts) {
      atomicAdd(&a.tier_counts[0], hits);
      atomicAdd(&a.tier_counts[1], misses);
    }
  }
}

__global__ void co_scatter_kernel(CoArgs c, const float* miss_d, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c.newk[c.miss_pos[i]] = make_key(miss_d[i], c.miss_id[i]);
}

__global__ __launch_bounds__(64) void co_merge_kernel(CoArgs c) {
  extern __shared__ __align__(16) unsigned char smem[];
  const SearchArgs& a = c.s;
  const int qi = blockIdx.x;
  const int lane = lane_id();
  const int n = c.newn[qi];
  if (n == 0) return;
  const int Lp = a.L_pow2;
  WaveCtx w;
  w.pool = reinterpret_cast<uint64_t*>(smem);
  w.next = w.pool + Lp;
  w.kept = w.next + Lp;
  w.L = a.L;
  w.ktrack = 0;
  uint64_t* gp = c.pool + (int64_t)qi * Lp;
  for (int i = lane; i < Lp; i += kWave) { w.pool[i] = gp[i]; w.next[i] = kKeyInf; }
  __syncthreads();
  const uint64_t* nk = c.newk + (int64_t)qi * c.C;
  for (int c0 = 0; c0 < n; c0 += kWave) {
    const uint64_t k = c0 + lane < n ? nk[c0 + lane] : kKeyInf;
    sort_merge(w, k);
  }
  for (int i = lane; i < Lp; i += kWave) gp[i] = w.pool[i];
}

__global__ void co_output_kernel(CoArgs c) {
  const SearchArgs& a = c.s;
  const int qi = blockIdx.x;
  const int lane = threadIdx.x;
  const uint64_t* gp = c.pool + (int64_t)qi * a.L_pow2;
  if (a.out_ids)
    for (int i = lane; i < a.k; i += blockDim.x) {
      const uint64_t pk = i < a.L ? gp[i] : kKeyInf;
      a.out_ids[(int64_t)qi * a.k + i] = key_id(pk);
      a.out_d[(int64_t)qi * a.k + i] = key_dist(pk);
    }
  if (lane == 0) {
    if (a.n_dist) a.n_dist[qi] = c.ndist[qi];
    if (a.n_exp) a.n_exp[qi] = c.iters[qi];
    if (a.trace_n) a.trace_n[qi] = c.iters[qi];
    if (a.totals) {
      atomicAdd(&a.totals[0], (unsigned long long)c.ndist[qi]);
      atomicAdd(&a.totals[1], (unsigned long long)c.iters[qi]);
    }
  }
}

// Host cores for the X_CPU distances: a fixed set of worker threads that
// split an index range in chunks.
class CpuPool {
 public:
  explicit CpuPool(int nt) {
    for (int i = 0; i < nt; ++i) workers_.emplace_back([this] { loop(); });
  }
  ~CpuPool() {
    {
      std::lock_guard<std::mutex> g(mu_);
      quit_ = true;
    }
    cv_work_.notify_all();
    for (auto& t : workers_) t.join();
  }
  void run(int64_t n, const std::function<void(int64_t, int64_t)>& fn) {
    std::lock_guard<std::mutex> one(run_mu_);
    std::unique_lock<std::mutex> lk(mu_);
    fn_ = &fn;
    n_ = n;
    next_ = 0;
    busy_ = (int)workers_.size();
    ++gen_;
    cv_work_.notify_all();
    cv_done_.wait(lk, [&] { return busy_ == 0; });
    fn_ = nullptr;
  }

 private:
  void loop() {
    uint64_t seen = 0;
    for (;;) {
      std::unique_lock<std::mutex> lk(mu_);
      cv_work_.wait(lk, [&] { return quit_ || gen_ != seen; });
      if (quit_) return;
      seen = gen_;
      const auto* fn = fn_;
      const int64_t n = n_;
      lk.unlock();
      constexpr int64_t kChunk = 256;
      for (;;) {
        const int64_t i = next_.fetch_add(kChunk);
        if (i >= n) break;
        (*fn)(i, std::min(n, i + kChunk));
      }
      lk.lock();
      if (--busy_ == 0) cv_done_.notify_one();
    }
  }
  std::vector<std::thread> workers_;
  std::mutex mu_, run_mu_;
  std::condition_variable cv_work_, cv_done_;
  const std::function<void(int64_t, int64_t)>* fn_ = nullptr;
  int64_t n_ = 0;
  std::atomic<int64_t> next_{0};
  int busy_ = 0;
  uint64_t gen_ = 0;
  bool quit_ = false;
};

CpuPool& cpu_pool() {
  static CpuPool p((int)std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
  return p;
}

}  // namespace

// The GPU gather's distance of one query row to one stored row, on the host:
// lane l of a 32-lane group holds elements c*128 + 4l + e (chunks c < nc,
// e < 4), each lane accumulates them in that order with fused multiply-adds,
// and the lanes are summed pairwise across distances 16, 8, 4, 2, 1.
float host_gather_dist(const float* q, const float* x, int dim, int64_t stride, int nc, int metric) {
  float p[32];
  for (int l = 0; l < 32; ++l) {
    float acc = 0.0f;
    for (int c = 0; c < nc; ++c) {
      const int64_t off = (int64_t)c * 128 + 4 * l;
      for (int e = 0; e < 4; ++e) {
        const int64_t idx = off + e;
        const float qv = idx < dim ? q[idx] : 0.0f;
        const float xv = off < stride ? x[idx] : 0.0f;
        if (metric == 0) {
          const float t = qv - xv;
          acc = std::fmaf(t, t, acc);
        } else {
          acc = std::fmaf(qv, xv, acc);
        }
      }
    }
    p[l] = acc;
  }
  for (int o = 16; o >= 1; o >>= 1) {
    float nxt[32];
    for (int l = 0; l < 32; ++l) nxt[l] = p[l] + p[l ^ o];
    for (int l = 0; l < 32; ++l) p[l] = nxt[l];
  }
  return metric == 0 ? p[0] : -p[0];
}

}  // namespace svf

namespace svf_detail {

// The co-processed search of nq device-resident queries (FP32 traversal over
// a tiered store); `a` is the filled argument block of the one-kernel search.
int co_search(svf_index* ix, const svf::SearchArgs& a, const float* d_q, int64_t nq, hipStream_t st) {
  svf::TierState& T = ix->tier;
  const int Lp = a.L_pow2;
  const int C = std::max(a.E, a.R);
  const int chunks = (int)((a.stride + 127) / 128);
  const int nc = chunks <= 1 ? 1 : chunks <= 2 ? 2 : chunks <= 4 ? 4 : 8;
  svf::CoArgs c{};
  c.s = a;
  c.C = C;
  int rc;
  int32_t* ints;
  float* missd;
  if ((rc = scratch_grow(T.co_pool, (size_t)nq * Lp, &c.pool)) ||
      (rc = scratch_grow(T.co_newk, (size_t)nq * C, &c.newk)) ||
      (rc = scratch_grow(T.co_ints, (size_t)nq * (4 + 2 * (size_t)C) + 2, &ints)) ||
      (rc = scratch_grow(T.co_missd, (size_t)nq * C, &missd)))
    return rc;
  c.state = ints;
  c.iters = ints + nq;
  c.ndist = ints + 2 * nq;
  c.newn = ints + 3 * nq;
  c.miss_pos = ints + 4 * nq;
  c.miss_id = c.miss_pos + nq * C;
  c.counters = c.miss_id + nq * C;
  CK(svf::launch_fill_u32(c.pool, (int64_t)nq * Lp * 2, 0xffffffffu, st));
  CK(svf::launch_fill_u32(ints, 4 * nq, 0u, st));
  // the queries on the host, for the X_CPU distances
  std::vector<float> qh((size_t)nq * ix->dim);
  CK(hipMemcpyAsync(qh.data(), d_q, qh.size() * 4, hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  const size_t lds_round = (size_t)Lp * 8 + 2 * svf::kWave * 4 + (size_t)std::max(a.E, 2 * Lp) * 4;
  const size_t lds_merge = (size_t)(2 * Lp + svf::kWave) * 8;
  std::vector<int32_t> mpos, mid;
  std::vector<float> md;
  for (int round = 0;; ++round) {
    CK(svf::launch_fill_u32(c.counters, 2, 0u, st));
    switch (nc) {
      case 1: hipLaunchKernelGGL(svf::co_round_kernel<1>, dim3((unsigned)nq), dim3(64), lds_round, st, c, round); break;
      case 2: hipLaunchKernelGGL(svf::co_round_kernel<2>, dim3((unsigned)nq), dim3(64), lds_round, st, c, round); break;
      case 4: hipLaunchKernelGGL(svf::co_round_kernel<4>, dim3((unsigned)nq), dim3(64), lds_round, st, c, round); break;
      default: hipLaunchKernelGGL(svf::co_round_kernel<8>, dim3((unsigned)nq), dim3(64), lds_round, st, c, round); break;
    }
    CK(hipGetLastError());
    int32_t cnt[2];
    CK(hipMemcpyAsync(cnt, c.counters, 8, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    const int32_t nmiss = cnt[0], nact = cnt[1];
    if (nmiss > 0) {
      mpos.resize(nmiss);
      mid.resize(nmiss);
      md.resize(nmiss);
      CK(hipMemcpyAsync(mpos.data(), c.miss_pos, (size_t)nmiss * 4, hipMemcpyDeviceToHost, st));
      CK(hipMemcpyAsync(mid.data(), c.miss_id, (size_t)nmiss * 4, hipMemcpyDeviceToHost, st));
      CK(hipStreamSynchronize(st));
      const int dim = ix->dim, metric = ix->metric;
      const int64_t stride = ix->stride;
      std::function<void(int64_t, int64_t)> job = [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
          const int64_t q = mpos[i] / C;
          md[i] = svf::host_gather_dist(qh.data() + q * dim, T.hrow(mid[i], stride), dim, stride,
                                        nc, metric);
        }
      };
      svf::cpu_pool().run(nmiss, job);
      CK(hipMemcpyAsync(missd, md.data(), (size_t)nmiss * 4, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(svf::co_scatter_kernel, dim3((unsigned)((nmiss + 255) / 256)), dim3(256), 0, st,
                         c, (const float*)missd, nmiss);
      CK(hipGetLastError());
    }
    if (nact == 0) break;
    hipLaunchKernelGGL(svf::co_merge_kernel, dim3((unsigned)nq), dim3(64), lds_merge, st, c);
    CK(hipGetLastError());
    T.co_rounds += 1;
  }
  hipLaunchKernelGGL(svf::co_output_kernel, dim3((unsigned)nq), dim3(64), 0, st, c);
  CK(hipGetLastError());
  return SVF_OK;
}

// Host-core time per distance of the co-processed miss path: the n rows
// ids[] of the host store against a zero query on the worker threads (one
// untimed run, then the median of five), in nanoseconds per row.
double host_distance_ns(svf_index* ix, const int32_t* ids, int n) {
  const int64_t stride = ix->stride;
  const int chunks = (int)((stride + 127) / 128);
  const int nc = chunks <= 1 ? 1 : chunks <= 2 ? 2 : chunks <= 4 ? 4 : 8;
  const svf::TierState& T = ix->tier;
  std::vector<float> q(stride, 0.0f), out(n);
  std::function<void(int64_t, int64_t)> job = [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i)
      out[i] = svf::host_gather_dist(q.data(), T.hrow(ids[i], stride), ix->dim, stride, nc,
                                     ix->metric);
  };
  svf::cpu_pool().run(n, job);
  std::vector<double> t;
  for (int r = 0; r < 5; ++r) {
    const auto t0 = std::chrono::steady_clock::now();
    svf::cpu_pool().run(n, job);
    t.push_back(std::chrono::duration<double, std::nano>(std::chrono::steady_clock::now() - t0).count());
  }
  std::sort(t.begin(), t.end());
  return t[2] / n;
}

}  // namespace svf_detail
