// Host-side state of one index handle.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <cmath>
#include <mutex>
#include <thread>
#include <string>
#include <vector>

#include "../../include/svf.h"
#include "kernels.hpp"
#include "mlp.hpp"
#include "wavp.hpp"

namespace svf {

// A device allocation that only grows.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // Make at least `need` bytes available; old contents are not kept.  A
  // reallocation takes `grow` bytes when that is more (room for later growth).
  hipError_t ensure(size_t need, size_t grow = 0) {
    if (need <= bytes && p) return hipSuccess;
    release();
    size_t b = need < 256 ? 256 : need;
    if (grow > b) b = grow;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) { p = nullptr; return e; }
    bytes = b;
    return hipSuccess;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// A pinned host allocation that only grows (old contents are not kept).
struct PinnedBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~PinnedBuf() { release(); }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
  }
  hipError_t ensure(size_t need) {
    if (need <= bytes && p) return hipSuccess;
    release();
    size_t b = need < 256 ? 256 : need + need / 4;
    hipError_t e = hipHostMalloc(&p, b, 0);
    if (e != hipSuccess) { p = nullptr; return e; }
    bytes = b;
    return hipSuccess;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

struct Options {
  uint64_t seed = 0;
  int beam_insert = 0;        // 0: 2 * degree
  int entry_samples = 0;
  int max_iters = 0;
  int search_width = 1;
  int coop_max_batch = 1024;
  int visited_slots = 0;        // 0: by traversal precision (visited_slots())
  int visited_compact = 1;
  int repair_c = 8;
  int localized_repair = 1;
  int consolidate_async = 0;
  int prune_cap = 0;
  double consolidate_frac = 0.2;
  int insert_batch_max = 10000;
  int precision = 0;
  int rerank = 1;
  // learned entry points / stopping step
  int use_model = 0;
  double model_conf = 0.5;
  double model_stop_scale = 1.5;
  int model_min_iters = 8;
  int model_entries = 1;        // 1: spread over the cluster, 0: nearest to the centroid
  int cache_cpu_miss = 0;       // tiered FP32 search: misses computed on the host cores
  int fp8_row_scales = -1;      // FP8 scales beside the rows: -1 by size, 0 off, 1 on
};

}  // namespace svf

namespace svf {
struct Server;

// Device buffers of one repair / consolidation pass.
// Workspace of the long-list kernels (candidate lists longer than the LDS
// kernels hold): raw keys, per-list offsets, hash tables, detour counts.
struct LongScratch {
  DevBuf keys, meta, hash, cnt, m, q;
  std::atomic<int64_t> lists{0};   // lists pruned here so far
};

struct RepairScratch {
  DevBuf list, cnt, rows, rows_d, cand, mcount, topup, topup_v, qkey, pool, qrows;
  LongScratch lg;
};

// A consolidation running in the background on a snapshot (Sec. 5.3): the
// snapshot's rows, edge distances and alive bits, the staged result, and
// the forward rows of the vertices inserted since the snapshot (their ids
// follow the snapshot's, in order) for the merge.
struct BgConsolidation {
  bool active = false;
  std::thread th;
  std::atomic<bool> done{false};
  int rc = 0;
  std::string err;
  hipStream_t st = nullptr;
  int64_t n0 = 0;
  int32_t n_aff = 0;
  DevBuf graph, edge_d, alive, mask;
  RepairScratch rs;
  DevBuf log_ids, log_d;
  int64_t log_n = 0, log_cap = 0;
};

// Tiered vector store: every vector lives in pinned host memory; an HBM cache
// of C rows, a device mapping table id -> slot, and the placement state.
// The host store is a list of pinned segments of 2^seg_shift rows (each one
// allocation, below the size one pinned allocation may take), so that it can
// grow segment by segment up to what pinned memory holds in all.
struct TierState {
  bool on = false;
  std::vector<float*> seg;         // host segments; the last may hold fewer rows
  std::vector<int64_t> seg_alloc;  // rows allocated per segment
  int seg_shift = 0;
  int64_t seg_rows_opt = 0;        // host_segment_rows option (0: by size)
  DevBuf seg_d;                    // device copy of seg (the kernels' table)
  int64_t C = 0;
  float* cache = nullptr;          // device, C x stride
  int32_t* map = nullptr;          // device, cap entries (-1 = not cached)
  std::vector<int32_t> slot_id;    // slot -> id (-1 empty)
  std::vector<int32_t> free_slots; // slots below `used` released by deletions (a stack)
  std::vector<int32_t> where;      // id -> slot (host mirror of map)
  std::vector<uint8_t> ref;        // reference bits per slot
  // F_recent per id as of batch `stamp` (the halvings of later batches are
  // applied on use); the two share a 16-byte record, one cache line fetch.
  struct FRec {
    double v = 0.0;
    int64_t stamp = 0;
  };
  std::vector<FRec> fr;
  // Per slot, a copy of fr of the slot's vector, kept in step with it (every
  // slot assignment goes through occupy(), and the per-batch update of a
  // cached vector writes both), so that the victim sweep reads it in slot
  // order instead of one scattered record per slot.
  std::vector<FRec> sfr;
  bool dead_residents = false;     // a deleted vector may hold a slot (deleted while serving)
  // Per slot, the in-degree of the slot's vector, likewise for the sweep:
  // rewritten from the device whenever the host copy of the in-degrees is,
  // and by occupy() in between.  Pinned when the host allows (sdeg_h), else
  // in ordinary memory (sdeg_v); sdeg points at the one in use.
  PinnedBuf sdeg_h;
  std::vector<int32_t> sdeg_v;
  int32_t* sdeg = nullptr;
  PinnedBuf e_in;                  // host copy: int32 in-degree per id, e_in_n of them
  int64_t e_in_n = 0;
  bool e_in_valid = false;         // e_in_d (cap entries) is kept current under updates
  int verify_indegree = 0;         // check the kept in-degrees against a recount
  int64_t used = 0, clock = 0, e_in_epoch = -1, batch = 0;
  int policy = 0;                  // 0 workload-aware (WAVP), 1 LRU, 2 LFU, 3 LRFU
  bool building = false;           // inside svf_build: the warm-up fills the cache afterwards
  std::vector<int64_t> freq;       // LFU: accesses so far per id
  std::vector<int64_t> last;       // LRU: last access, (batch << 40) + position, -1 never
  double alpha = 0.6, beta = 0.4, theta = 1.0;
  // theta adaptation (Sec. 4.4): factor (0 = off), the starting theta, and
  // the miss rate and mean missed prediction of the last batch with accesses
  double adapt = 0.0, theta0 = 1.0, prev_mean = 0.0;
  bool have_prev = false;
  int64_t prev_miss = 0, prev_acc = 0;
  WavpSweep sweep;                 // Alg. 2's victim choice within a batch
  int promote_max = 2048, trace_cap = 512;
  uint64_t gather_hits = 0, gather_misses = 0, promotions = 0, evictions = 0;
  int64_t last_trace_hits = 0, last_placed = 0;
  // co-processed search (misses computed on the host cores): per-batch pools,
  // round keys, miss lists, and the rounds run so far
  DevBuf co_pool, co_newk, co_ints, co_missd;
  int64_t co_rounds = 0;
  DevBuf trace, trace_n, place, counts, e_in_d, acc_cnt, touched, lastpos, sdeg_d;
  DevBuf blk, lst_id, lst_cnt, lst_last;   // the batch's touched vertices, in id order
  DevBuf e_in_chk;                         // recount for cache_indegree_verify
  PinnedBuf blk_h, lst_id_h, lst_cnt_h, lst_last_h, alive_h;
  // A free slot (released ones first, then the untouched tail), -1 when full.
  // Slot `slot` now holds vector x, with a clear reference bit.
  void occupy(int64_t slot, int32_t x) {
    slot_id[slot] = x;
    where[x] = (int32_t)slot;
    ref[slot] = 0;
    sfr[slot] = fr[x];
    sdeg[slot] = x < e_in_n ? in_degree(x) : 0;   // refreshed with the in-degrees
  }
  int64_t take_slot() {
    if (!free_slots.empty()) {
      const int64_t s = free_slots.back();
      free_slots.pop_back();
      return s;
    }
    return used < C ? used++ : -1;
  }
  int64_t free_count() const { return (int64_t)free_slots.size() + (C - used); }
  // host address of row id of the segmented store
  float* hrow(int64_t id, int64_t stride) const {
    return seg[(size_t)(id >> seg_shift)] + (id & ((int64_t(1) << seg_shift) - 1)) * stride;
  }
  HostSegs segs() const { return HostSegs{seg_d.as<const float* const>(), seg_shift}; }
  int32_t in_degree(int32_t x) const { return e_in.as<int32_t>()[x]; }
  // log(1 + e) for in-degree e, from a table of the same values for small e
  std::vector<double> log1p_tab;
  double log1p_deg(int32_t e) {
    if (log1p_tab.empty()) {
      log1p_tab.resize(1 << 16);
      for (int i = 0; i < (1 << 16); ++i) log1p_tab[i] = std::log(1.0 + (double)i);
    }
    return (uint32_t)e < log1p_tab.size() ? log1p_tab[e] : std::log(1.0 + (double)e);
  }
};
}  // namespace svf

struct svf_index {
  int dim = 0, R = 0, metric = 0;
  int64_t stride = 0;                // stored row length in elements (multiple of 8)
  int64_t cap = 0, n_slots = 0, n_alive = 0;
  int device = 0;
  // device-resident state
  float* vec32 = nullptr;            // cap x stride FP32
  void* veclp = nullptr;             // reduced-precision traversal store (FP16/BF16 rows, or FP8
                                     // rows then per-vector scales)
  int veclp_prec = 0;
  int32_t* graph = nullptr;          // cap x R
  float* nscale = nullptr;           // FP8: cap x R scales of the vectors the rows name (or null)
  float* edge_d = nullptr;           // cap x R
  uint32_t* alive = nullptr;         // ceil(cap/32) words
  svf::Options opt;
  int64_t deleted_since = 0, alive_at_consolidate = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::mutex mu;
  // scratch
  svf::DevBuf s_q, s_qkey, s_ids, s_d, s_pool, s_tot, s_misc[12];
  svf::DevBuf s_rows;                // FP32 rows staged in HBM for a tiered store's kernels
  // learned form
  svf::Mlp* model = nullptr;
  int model_nc = 0, entry_cap = 0;
  svf::DevBuf centroids, entry_lists, s_z, s_qentry, s_qmax;
  svf_stats st{};
  svf::Server* server = nullptr;   // non-null while the serving loop runs
  svf::TierState tier;
  svf::RepairScratch rs;             // foreground repair / consolidation
  svf::LongScratch lrev;             // long reverse-edge lists (insertion, merge)
  svf::BgConsolidation bg;
  int64_t graph_epoch = 0;         // advances whenever rows are committed
};
