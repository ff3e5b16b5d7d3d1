// Launch interfaces of the library's HIP kernels (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace svf {

// Rows of the tiered FP32 store: pinned host memory in segments of 2^shift
// rows, segment i holding rows [i << shift, (i + 1) << shift).  seg is a
// device-readable table of the segment bases (null: no segments).
struct HostSegs {
  const float* const* seg;
  int shift;
  __device__ __forceinline__ const float* row(int32_t id, int64_t stride) const {
    const uint32_t u = (uint32_t)id;
    return seg[u >> shift] + (int64_t)(u & ((1u << shift) - 1u)) * stride;
  }
};

struct SearchArgs {
  // index snapshot
  const void* vec;          // traversal store: FP32 / FP16 / BF16 / FP8, n x vstride
  const float* vec32;       // exact FP32 store (re-scoring), n x stride
  int64_t stride;           // elements per FP32 row (multiple of 8)
  int64_t vstride;          // elements per traversal row (0: stride; FP8: multiple of 16)
  const float* vscale;      // FP8: per-vector scales
  const float* nscale;      // FP8 (optional): per row entry, the scale of the vector it names,
                            // n x R beside graph; the search then reads no per-vector scale
  int dim;
  const int32_t* graph;     // n x R ids
  int R;
  const uint32_t* alive;    // deletion bitset (1 = alive)
  int32_t n_slots;          // ids in [0, n_slots) exist in the snapshot
  int32_t n_alive;
  int metric;               // 0 = squared L2, 1 = -inner product
  // search parameters
  int L, L_pow2, k, E, max_iters, T, rerank;
  int width;                // parents expanded per iteration (1..4)
  int coop_max_nq;          // batches up to this size run width 2 or 4 with one wave per
                            // parent (0: never)
  int vis_compact;          // allow 16-bit visited tags when ids fit
  int id_bits;              // set by the launcher
  // queries
  const float* queries;     // FP32 rows, qstride apart
  int64_t qstride;
  const int32_t* qids;      // optional: query i is row qids[i] of `queries`
  const uint64_t* qkey;     // per-query entry stream keys
  int nq;
  // outputs (any may be null)
  int32_t* out_ids;         // nq x k
  float* out_d;             // nq x k
  uint64_t* out_pool;       // nq x L final pool keys (flag cleared)
  int32_t* n_dist;
  int32_t* n_exp;
  // learned entry points and stopping steps (all optional)
  const int32_t* entry_lists;  // nlists x entry_cap ids (-1 padded)
  int entry_cap;
  const int32_t* q_entry;      // per query: list index, or -1 for random entries
  const int32_t* q_max_iters;  // per query iteration cap (0: none)
  int32_t* last_change;        // per query: iterations done when the top-k last changed
  // tiered vector store: the FP32 rows sit in host segments (hsegs; vec and
  // vec32 are then unused), an FP32 traversal reads through the cache
  HostSegs hsegs;
  const int32_t* tmap;         // id -> HBM cache slot, -1 when not cached
  const float* tcache;         // cache rows, stride apart
  int32_t* trace;              // per query: expanded vertices in order (trace_cap each)
  int trace_cap;
  int32_t* trace_n;            // per query: number of expansions
  unsigned long long* tier_counts;  // [0] gathers from the cache, [1] from the host store
  unsigned long long* totals;  // [0] distances, [1] expansions
};

hipError_t launch_search(const SearchArgs& a, int precision, hipStream_t st);
bool coop_eligible(const SearchArgs& a, int precision, int nc);
hipError_t launch_search_coop(const SearchArgs& a, int precision, int nc, bool tags, size_t vis,
                              hipStream_t st);
hipError_t launch_query_keys(const float* q, int64_t qstride, const int32_t* qids, int dim, int nq,
                             uint64_t seed, uint64_t* out, hipStream_t st);

// ---- tiered store (tier.hip) ----
hipError_t launch_indegree(const int32_t* graph, const uint32_t* alive, int64_t n, int R,
                           int32_t* e_in, hipStream_t st);
hipError_t launch_place(const int32_t* place, int np, HostSegs store, float* cache,
                        int64_t stride, int32_t* map, hipStream_t st);
// sdeg[map[i]] = e_in[i] for every id i < n that holds a slot
hipError_t launch_slot_indegree(const int32_t* map, const int32_t* e_in, int64_t n, int32_t* sdeg,
                                hipStream_t st);
int64_t touched_blocks(int64_t words);
// rows: an HBM array (hs.seg null) or the host segments
hipError_t launch_probe_gather(const float* rows, HostSegs hs, const int32_t* idx, int n,
                               int64_t stride, int dim, const float* q, float* out, hipStream_t st);
// Listed rows of the host segments copied into dst (n rows, stride apart).
hipError_t launch_gather_rows(HostSegs store, const int32_t* idx, int n, int64_t stride,
                              float* dst, hipStream_t st);
hipError_t launch_touched_count(const uint32_t* touched, int64_t words, int32_t* block_tot,
                                hipStream_t st);
hipError_t launch_touched_list(const uint32_t* touched, int64_t words, const int32_t* block_off,
                               const int32_t* cnt, const int32_t* lastpos, int32_t* out_id,
                               int32_t* out_cnt, int32_t* out_last, hipStream_t st);
hipError_t launch_trace_count(const int32_t* trace, const int32_t* trace_n, int nq, int cap,
                              int32_t* cnt, uint32_t* touched, int32_t* lastpos, hipStream_t st);

// ---- index maintenance (update.hip) ----
hipError_t launch_fill_u32(void* p, int64_t n, uint32_t v, hipStream_t st);
// Reduced-precision rows [row0, row0 + nrows) of the traversal store from the
// FP32 rows at src (row row0 first, stride apart).
hipError_t launch_store_lowp(const float* src, int64_t stride, int dim, void* veclp,
                             int64_t lp_stride, float* vscale, int64_t row0, int64_t nrows,
                             int precision, hipStream_t st);
hipError_t launch_seed(const float* vec32, int64_t stride, int dim, int metric, int s0, int R,
                       int32_t* graph, float* edge_d, hipStream_t st);
hipError_t launch_set_alive(uint32_t* alive, int64_t lo, int64_t hi, hipStream_t st);
// nscale[v * R + r] = vscale[graph[v * R + r]] (0 for an empty entry) for the
// rows v of list[0, n), or, with list null, for rows [lo, lo + n).
hipError_t launch_row_scales(const int32_t* graph, int R, const int32_t* list, int64_t lo, int64_t n,
                             const float* vscale, float* nscale, hipStream_t st);

struct PruneArgs {
  const uint64_t* cand;     // lists of sorted keys, cstride apart (kKeyInf padded)
  int cstride;
  int cap;                  // at most this many candidates per list are pruned
  const int32_t* graph;     // rows of ids < n_old
  const int32_t* fwd;       // rows of ids >= n_old (staged rows of a batch)
  int32_t n_old;
  int R;
  int32_t* out_ids;         // nlists x R
  float* out_d;
  int nlists;
  const int32_t* skip;      // optional: lists with skip[l] < 0 are left alone
};
size_t prune_lds_bytes(int cap);
hipError_t launch_prune_lists(const PruneArgs& a, hipStream_t st);

// ---- candidate lists longer than the LDS kernels hold (longprune.hip) ----
// List l's raw keys are keys[off[l], off[l+1]) (any order, repeats allowed,
// at most kLongMaxKeys).  The host lays out, per list, a hash table of
// 2 * S_l words at hoff[l] (S_l a power of two >= 2 * its raw length; hoff
// has n + 1 entries) and 2 * len_l + 1 count words at coff[l].  Row l of the
// output is written at out + dst[l] * R.
constexpr int kLongMaxKeys = 16384;
struct LongLists {
  int n;
  const int64_t* off;       // n + 1
  const int64_t* hoff;      // n + 1, in 32-bit words
  const int64_t* coff;      // n, in 32-bit words
  const int32_t* dst;       // n
  uint64_t* keys;           // raw keys; sorted distinct keys after launch_long_sort
  int32_t* m;               // distinct candidates per list
  int skip_m;               // launch_long_prune leaves lists of at most skip_m alone
  uint32_t* hash;
  uint32_t* cnt;
};
struct LongRows {
  const int32_t* graph;     // rows of ids < n_old
  const int32_t* fwd;       // rows of ids >= n_old (staged rows of a batch)
  int32_t n_old;
  int R;
};
hipError_t launch_long_sort(const LongLists& a, int max_len, hipStream_t st);
hipError_t launch_long_prune(const LongLists& a, const LongRows& rs, int32_t* out_ids, float* out_d,
                             int64_t hash_words, int64_t cnt_words, hipStream_t st);

struct ReverseArgs {
  const int32_t* fwd_ids;   // b x R forward rows of the batch
  const float* fwd_d;
  int b, R;
  int32_t n0;               // first id of the batch
  int32_t* tcount;          // per-vertex incoming counts (cap entries, zero outside a batch)
  int32_t* tidx;            // per-vertex index into the target list
  int32_t* tlist;           // targets (b x R max)
  int32_t* n_targets;       // device counter
  int32_t* off;             // n_targets + 1 offsets
  int32_t* cursor;          // n_targets
  uint64_t* inc;            // incoming keys grouped by target
  const int32_t* graph;
  const float* edge_d;
  const uint32_t* alive;
  int cap;
  int32_t* trow;            // n_targets x R
  float* trow_d;
  const uint32_t* tmask;    // only targets with their bit set take edges (null: all)
  int32_t rows_below;       // the prune reads rows of ids below this from graph (0: n0)
  int32_t* long_q;          // optional: targets with more than cap candidates are queued here
  int32_t* long_len;        // (index k, list length) instead of being pruned
  int32_t* long_n;
};
hipError_t launch_reverse_count(const ReverseArgs& a, hipStream_t st);
hipError_t launch_reverse_scan_scatter(const ReverseArgs& a, int n_targets, hipStream_t st);
hipError_t launch_reverse_prune(const ReverseArgs& a, int n_targets, hipStream_t st);
hipError_t launch_commit_batch(const ReverseArgs& a, int n_targets, int32_t* graph, float* edge_d,
                               uint32_t* alive, hipStream_t st);

struct RepairArgs {
  const float* vec32;
  HostSegs hsegs;           // tiered store: the FP32 rows (vec32 unused)
  int64_t stride;
  int dim, metric, R;
  const int32_t* graph;
  const float* edge_d;
  const uint32_t* alive;
  int32_t n_slots;
  int consolidate;          // 0: more than half deleted, c = repair_c; 1: any deleted, c = R
  int c;
  int cap;
  int32_t* list;            // affected vertices
  int32_t* n_list;          // device counter
  uint64_t* cand;           // nlist x cap
  int32_t* mcount;          // nlist
  int32_t* topup;           // chunk-local indices needing a search top-up
  int32_t* topup_v;         // their vertex ids
  int32_t* n_topup;
  int32_t* over_li;         // chunk-local indices of lists that offered more than cap keys
  int32_t* over_len;        // their offered key counts (null over_li: no queue)
  int32_t* n_over;
};
hipError_t launch_mark_deleted(const int32_t* ids, int64_t n, uint32_t* alive, int32_t* newly,
                               const int32_t* graph, int R, int32_t* e_in, hipStream_t st);
hipError_t launch_indegree_rows_delta(const int32_t* graph, const int32_t* list, int n,
                                      const int32_t* rows, int R, int32_t* e_in, hipStream_t st);
hipError_t launch_indegree_add(const int32_t* rows, int64_t n, int32_t* e_in, hipStream_t st);
hipError_t launch_mark_list(const int32_t* list, int n, uint32_t* mask, hipStream_t st);
hipError_t launch_affected(const RepairArgs& a, hipStream_t st);
hipError_t launch_repair_candidates(const RepairArgs& a, int first, int count, hipStream_t st);
// The walk of launch_repair_candidates for the L.n queued lists (a.over_li),
// writing every offered key to L.keys + L.off[l].
hipError_t launch_repair_raw(const RepairArgs& a, int first, const LongLists& L, hipStream_t st);
hipError_t launch_repair_back(const RepairArgs& a, int first, const LongLists& L, hipStream_t st);
hipError_t launch_reverse_gather(const ReverseArgs& a, const int32_t* qk, const LongLists& L,
                                 hipStream_t st);
hipError_t launch_topup_merge(const RepairArgs& a, const uint64_t* pool, int L, int first,
                              int ntop, hipStream_t st);
hipError_t launch_commit_rows(const int32_t* list, int n, const int32_t* rows, const float* rows_d,
                              int R, int32_t* graph, float* edge_d, hipStream_t st);

}  // namespace svf
