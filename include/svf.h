/*
 * svf.h -- C ABI of the MI355X streaming graph-ANN library.
 *
 * The library keeps one proximity-graph index per handle entirely in the
 * GPU's HBM and runs every step of search, insertion, deletion and repair in
 * hand-written HIP kernels for gfx950.  The operations follow the streaming
 * ANNS problem statement of SVFusion (arXiv 2601.08528, Sec. 2.2): Build,
 * Search(q, k), Insert(x) and Delete(x) evolve a dataset state one operation
 * (here: one batch) at a time.
 *
 * Conventions shared by every call
 *  - Every function returns an int status (SVF_OK or a negative SVF_E_* code);
 *    no C++ exception crosses this boundary.  svf_last_error() gives a
 *    message for the last failure on the calling thread.
 *  - Ids are dense int32 numbers assigned in insertion order from 0 and never
 *    reused.  INVALID ids are -1.
 *  - Distances are squared Euclidean for SVF_METRIC_L2 (the ranking of the
 *    paper's L2 norm, Sec. 2.1) and -<q,x> for SVF_METRIC_IP.
 *  - Ordering is by the key (distance, id), lexicographically.
 *  - Host-pointer calls copy their inputs before returning and block until
 *    their outputs are written.  The caller owns every buffer.
 *  - *_dev calls take device pointers and a hipStream_t (passed as void *,
 *    NULL = the handle's own stream); they enqueue work on that stream and
 *    return without waiting, unless noted.
 *  - A failed call leaves the index as it was; outputs are then undefined.
 *  - Calls on one handle are serialised by the library.
 */
#ifndef SVF_H
#define SVF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct svf_index svf_index;

enum { SVF_METRIC_L2 = 0, SVF_METRIC_IP = 1 };

enum {
    SVF_OK = 0,
    SVF_E_INVAL = -1,     /* bad argument or option value                   */
    SVF_E_NOMEM = -2,     /* device memory exhausted (index unchanged)      */
    SVF_E_DEVICE = -3,    /* HIP runtime error                              */
    SVF_E_NOTFOUND = -4,  /* an id outside [0, n_slots)                     */
    SVF_E_BUSY = -5,      /* serving loop state does not allow the call     */
    SVF_E_INTERNAL = -6
};

/* Precision of the distances evaluated during graph traversal.  Reduced
 * precision keeps an FP16 / BF16 copy of every vector, computes in FP32, and
 * re-scores the final candidate pool with exact FP32 distances. */
enum { SVF_PREC_FP32 = 0, SVF_PREC_FP16 = 1, SVF_PREC_BF16 = 2, SVF_PREC_FP8 = 3 };

typedef struct svf_stats {
    int64_t n_slots;          /* ids assigned so far                          */
    int64_t n_alive;          /* ids not deleted                              */
    int64_t capacity;         /* id slots allocated on the device             */
    /* last search call (sums over its queries) */
    int64_t last_queries;
    int64_t last_n_dist;      /* distance evaluations                         */
    int64_t last_n_exp;       /* expanded vertices (graph rows read)          */
    double last_search_ms;    /* device time of the search kernels            */
    /* last insert / delete call, device time per phase (ms) */
    double ins_search_ms, ins_prune_ms, ins_reverse_ms, ins_commit_ms;
    double del_mark_ms, del_repair_ms;
    int64_t last_repaired;    /* rows rewritten by the last delete/consolidate */
    int64_t device_bytes;     /* HBM held by the index                        */
    /* tiered store (cache_bytes set) */
    int64_t cache_slots;            /* vectors the HBM cache holds            */
    int64_t cache_gather_hits;      /* search gathers served by the cache     */
    int64_t cache_gather_misses;    /* search gathers read from host memory   */
    int64_t cache_last_trace_hits;  /* last batch: expansions of cached vectors */
    int64_t cache_last_placed;      /* last batch: vectors placed in the cache */
    int64_t cache_promotions, cache_evictions;
    int64_t consolidations;         /* global consolidations done (a background one once merged) */
    int64_t last_model_fallback;    /* last search with use_model: queries below model_conf that
                                       ran plain search */
    int64_t long_lists;             /* candidate lists so far too long for the one-wave LDS
                                       prune, pruned whole by the long-list kernels */
    /* tiered store: host-clock time of the last batch's placement (ms), by phase */
    double place_count_ms;   /* access counts and touched list on the GPU, copied back   */
    double place_indeg_ms;   /* in-degrees brought up to date (after the graph changed)  */
    double place_walk_ms;    /* F_recent, hits and candidates over the touched vertices */
    double place_evict_ms;   /* Alg. 2's victims, scoring the residents included        */
    double place_apply_ms;   /* rows copied into the cache and the map rewritten         */
} svf_stats;

/* Create an empty index.  Sec. 2.3: a directed graph with a fixed number of
 * out-edges (degree) per vertex.  dim >= 1 and <= 1024; 1 <= degree <= 128;
 * metric is SVF_METRIC_L2 or SVF_METRIC_IP.  *out receives the handle.
 * Allocates a small initial capacity on the current HIP device. */
int svf_create(int32_t dim, int32_t degree, int32_t metric, svf_index **out);

/* Release the handle and all its device memory.  NULL is accepted. */
int svf_destroy(svf_index *ix);

/* Set a numeric option.  Keys (range; default):
 *   seed            entry-point hash seed (any; 0)
 *   beam_insert     candidate pool size of the insertion search (degree..512; 2*degree)
 *   entry_samples   random entry points per query, 0 = the pool size (0..1024; 0)
 *   max_iters       cap on iterations per query, 0 = none (>= 0; 0)
 *   search_width    parents expanded per iteration (1..4; 1)
 *   coop_max_batch  with search_width 2 or 4, batches of at most this many queries run
 *                   one wave per parent, the waves of a query sharing its pool (results
 *                   unchanged; FP32/BF16/FP8, degree <= 64, dim <= 256, untiered)
 *                   (0..2^22; 1024; 0 = never)
 *   visited_slots   LDS visited-table slots per query: a power of two (256..16384), or 0
 *                   for 4096 with FP32 traversal and 2048 with reduced precision on up to
 *                   2^24 ids (0; the size never changes results, only re-evaluations
 *                   against occupancy)
 *   visited_compact exact quotient tags of a scrambled id (12-bit, five per 64-bit set, or
 *                   16-bit, four per set) instead of full 32-bit ids, when the ids fit (0/1; 1)
 *   repair_c        out-neighbours taken from each deleted neighbour (1..min(16, degree); 8)
 *   prune_cap       0 (the method): every candidate list is pruned whole (Sec. 5.1, 5.2),
 *                   up to 16384 candidates per list; > 0: an experiment that cuts each list to
 *                   its prune_cap nearest candidates first (0..; 0)
 *   consolidate_frac deleted fraction that triggers consolidation ([0,1]; 0.2; 0 = never)
 *   localized_repair repair the affected vertices after each deletion (0/1; 1).  With 0
 *                   and consolidate_frac 0 deletion is lazy only (the paper's ablation)
 *   consolidate_async run a consolidation that falls due in the background on a snapshot
 *                   and merge it later (svf_consolidate_wait) (0/1; 0; with a tiered
 *                   store consolidation stays synchronous)
 *   insert_batch_max largest batch of one insertion pass (1..1<<20; 10000)
 *   precision       SVF_PREC_* of traversal distances (0..3; 0).  FP16/BF16: each element
 *                   rounded to nearest even.  FP8: OCP E4M3 codes of x / s with one FP32
 *                   scale s = max|x| / 448 per vector (the query quantised the same way);
 *                   distances accumulate in FP32
 *   rerank          exact FP32 re-scoring of the final pool under reduced precision (0/1; 1)
 *   fp8_row_scales  FP8 traversal: keep, beside every graph row, the scales of the vectors it
 *                   names (capacity x degree floats in HBM, refreshed for every row written),
 *                   so the search reads a row's scales with its ids instead of one scattered
 *                   4-byte scale per distance; results are identical.  -1 = when the index
 *                   holds 2^24 vectors or more, 0 = off, 1 = on (-1, 0, 1; -1).  Read-only
 *                   "fp8_row_scales_on" tells whether the scales are kept now
 *   capacity        reserve id slots for this many vectors now (never shrinks); otherwise
 *                   the stores grow by reallocation to twice their size when full, which
 *                   briefly holds both copies (1..2^31-65)
 *   cache_bytes     tiered store (Sec. 4.2-4.3): all FP32 vectors in pinned host memory, an
 *                   HBM cache of cache_bytes / (4 * round_up(dim, 8)) rows in front.  An FP32
 *                   traversal reads through the cache; with FP16/BF16/FP8 traversal that
 *                   store stays in HBM and only the exact re-scoring reads go through the
 *                   cache.  Set on an empty index, or on a filled one (its vectors
 *                   then move to host memory and the cache is warmed by in-degree, as
 *                   after svf_build).  Once set it stays.  Searches read cached rows from HBM
 *                   and the rest over the host link; after every direct search call the
 *                   batched workload-aware placement (Alg. 2) updates the cache, and
 *                   svf_build warms it with the highest in-degree vectors (Sec. 4.4).
 *                   A deleted vector leaves the cache at once; inserted vectors take
 *                   free slots in id order.  While the serving loop runs the cache
 *                   does not change.  The host store is a set of pinned segments of
 *                   host_segment_rows rows each (one allocation per segment), so it
 *                   grows segment by segment up to what pinned memory holds in all.
 *                   svf_model_fit is refused once the store is tiered
 *   host_segment_rows rows per pinned host segment of the tiered store, set before
 *                   cache_bytes: 0 = the most rows whose segment stays within 4 GiB
 *                   (at least 4096), else a power of two in [1024, 2^30] (0).  Reading it
 *                   back once tiered gives the size in force; "host_segments" (read-only)
 *                   is the number of segments
 *   cache_theta     placement threshold on F_lambda (>= 0; 1.0); also the floor of the
 *                   adaptation below.  svf_cache_calibrate sets it from measured costs
 *   cache_theta_adapt Sec. 4.4's adaptation of theta, by this factor, 0 = off (0 or (1, 16];
 *                   0): after a batch's accesses are counted, its miss rate and the mean
 *                   F_lambda of its distinct missed alive vectors are compared with the last
 *                   batch's; both higher multiplies theta by the factor, both lower divides
 *                   it (not below cache_theta); the value in force is readable as cache_theta
 *   cache_alpha_ratio alpha / (alpha + beta) of F_lambda, alpha + beta = 1 ([0,1]; 0.6)
 *   cache_promote_max placements per query batch (>= 0; 2048)
 *   cache_trace_cap expansions per query recorded for placement (16..8192; 512)
 *   cache_cpu_miss  Alg. 1's co-processing (0/1; 0): an FP32 traversal of the tiered store
 *                   computes the distances of uncached neighbours on the host cores (X_CPU)
 *                   and those of cached ones on the GPU (X_GPU), round by round over the
 *                   batch; 0 reads uncached rows over the host link inside the search kernel.
 *                   Results are identical either way (the host follows the GPU's FP32
 *                   summation order).  Applies to svf_search / svf_search_dev with random
 *                   entry points and search_width 1; other searches keep the one-kernel form.
 *                   The read-only key cache_cpu_rounds counts the rounds run so far
 *   cache_policy    placement policy: 0 workload-aware (Alg. 2), or one of the classic
 *                   policies the paper compares it with, in the same batched form:
 *                   1 LRU, 2 LFU, 3 LRFU (0..3; 0)
 *   use_model       learned entry points and stopping step (0/1; 0; needs svf_model_fit)
 *   model_conf      softmax confidence below which a query falls back to plain search ([0,1]; 0.5)
 *   model_stop_scale expansion cap = ceil(scale * predicted stop step) (>0; 1.5)
 *   model_min_iters smallest expansion cap of a gated query (>=1; 8)
 *   model_entries   how svf_model_fit fills a cluster's entry list: 1 = spread over the
 *                   cluster's members (evenly through its members in the clustered sample,
 *                   so every part of the cluster holds entries), 0 = the vectors nearest
 *                   to its centroid (0/1; 1)
 * Unknown key or out-of-range value: SVF_E_INVAL. */
int svf_set_option(svf_index *ix, const char *key, double value);
/* Any key above, plus the read-only "dim", "degree", "metric" and
 * "cache_resident" (vectors currently held in the HBM cache). */
int svf_get_option(const svf_index *ix, const char *key, double *value);

/* Insert n vectors (n x dim row-major FP32, host memory) as one batch
 * (Sec. 5.1): each new vector searches the pre-batch graph for candidates,
 * keeps the rank-based reordering of them as its out-edges, and its chosen
 * neighbours receive reverse edges.  Batches larger than insert_batch_max are
 * split.  out_ids (n entries, may be NULL) receives the assigned ids.
 * Non-finite input: SVF_E_INVAL. */
int svf_insert(svf_index *ix, const float *vecs, int64_t n, int32_t *out_ids);
/* Same with device pointers.  Waits for the work already queued on `stream`
 * (the producer of d_vecs; NULL is the default stream), runs on the index's
 * own stream and has finished when it returns. */
int svf_insert_dev(svf_index *ix, const float *d_vecs, int64_t n, int32_t *d_out_ids, void *stream);

/* Build from scratch by the insertion rule: the first min(n, 4*degree)
 * vectors form an exact nearest-neighbour seed graph, the rest are inserted in
 * batches of min(insert_batch_max, ceil(n_alive / 8)).  The index must be
 * empty.  vecs: host memory. */
int svf_build(svf_index *ix, const float *vecs, int64_t n);

/* Delete ids (Sec. 5.2): mark them in the deletion bitset, then repair every
 * alive vertex with more than half of its neighbours deleted from at most
 * repair_c out-neighbours of each deleted neighbour; consolidate when the
 * deleted fraction since the last consolidation reaches consolidate_frac.
 * An id outside [0, n_slots) gives SVF_E_NOTFOUND and no change; deleting an
 * id twice is harmless.  ids: host memory. */
int svf_delete(svf_index *ix, const int32_t *ids, int64_t n);

/* Global consolidation (Sec. 5.2): rebuild every alive row that names a
 * deleted vertex.  Afterwards no edge points at a deleted id.  A pending
 * background consolidation is merged first. */
int svf_consolidate(svf_index *ix);
/* With consolidate_async = 1, a consolidation that falls due during a delete
 * runs in the background (Sec. 5.3): on a snapshot of the graph taken then,
 * on a stream and host thread of its own, while calls continue on the live
 * graph (insertions are logged; deletions repair locally; a consolidation
 * that falls due meanwhile waits for this one).  svf_consolidate_wait blocks
 * until it has finished and merges it into the live graph: the consolidated
 * rows are written, then each of them is re-pruned with the reverse edges
 * that insertions since the snapshot gave it.  Rows of vertices inserted
 * since, and rows the consolidation did not rewrite, keep their live state.
 * No-op when nothing is pending; the serving loop merges by itself
 * (SVF_E_BUSY while serving).  A failure of the background pass is reported
 * here.  svf_get_option(ix, "consolidate_pending") tells whether one is. */
int svf_consolidate_wait(svf_index *ix);

/* Batched search (Sec. 4.2, Algorithm 1): for each of nq queries (nq x dim
 * FP32, host memory) a best-first search with a candidate pool of `beam`
 * entries (k <= beam <= 1024) from random entry points, stopping when every
 * pool entry is expanded; the k nearest found are written to out_ids and
 * out_dists (nq x k each, ascending).  Fewer than k alive vectors: the rest
 * is padded with id -1 and distance +inf.  nq <= 2^25 per call (SVF_E_INVAL
 * beyond). */
int svf_search(svf_index *ix, const float *queries, int64_t nq, int32_t k, int32_t beam,
               int32_t *out_ids, float *out_dists);

/* Device-pointer search, enqueued on `stream` (NULL is the default stream)
 * after the work already queued there, without waiting for it to finish
 * (with a tiered store the call waits, since placement follows the batch).
 * The index's scratch buffers serve one search at a time: a search on another
 * stream must not start before this one has finished.  Optional d_n_dist /
 * d_n_exp (nq int32 each, may be NULL) receive per-query counts of distance
 * evaluations and expanded vertices. */
int svf_search_dev(svf_index *ix, const float *d_queries, int64_t nq, int32_t k, int32_t beam,
                   int32_t *d_out_ids, float *d_out_dists, int32_t *d_n_dist, int32_t *d_n_exp,
                   void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * search as svf_search_dev, with the same arguments, outputs and stream
 * semantics, that calls no hipMalloc, hipFree or other allocating routine.
 * Its only workspace, one 8-byte entry-stream key per query, lives in a
 * fixed 4 MiB array of device memory that every GPU the library runs on
 * holds until the process ends, so nq is limited to 524,288 (SVF_E_INVAL
 * beyond).  All calls on one GPU share that array, across indexes: calls
 * that overlap on one GPU (on different streams, or from different threads)
 * race on it and must be ordered by the caller.  Refused with SVF_E_INVAL
 * when the learned form (use_model) or a tiered store is on, since those
 * need more workspace; the batch totals that svf_stats_get reports
 * (last_n_dist, last_n_exp) are not updated by this call (the per-query
 * counts d_n_dist / d_n_exp are). */
int svf_search_dev_noalloc(svf_index *ix, const float *d_queries, int64_t nq, int32_t k,
                           int32_t beam, int32_t *d_out_ids, float *d_out_dists,
                           int32_t *d_n_dist, int32_t *d_n_exp, void *stream);

/* Learned entry points and stopping step (an extension of the method: the
 * paper starts from random entry points, Sec. 4.2, and notes that entry
 * points may come from a separate algorithm, Sec. 2.3).  Trains, on the GPU,
 * a predictor din -> 256 -> 256 -> (n_clusters + 1) with BF16 weights and
 * FP32 accumulation on search traces this index produces:
 *   1. Lloyd k-means (12 iterations) of an evenly spaced sample of at most
 *      65,536 stored vectors into n_clusters centroids;
 *   2. plain search of the n training queries (host memory, n x dim FP32)
 *      with k and beam, recording each query's top-1 id and the expansion
 *      count after which its top-k stopped changing;
 *   3. labels: the centroid nearest to the top-1 vector, and log(max(1, step));
 *   4. per cluster, an entry list of 64 stored vectors: spread over the
 *      cluster's alive members in the sample (model_entries = 1), or the
 *      64 nearest stored vectors to its centroid (model_entries = 0);
 *   5. Adam over epochs/2 passes of batches of 1024, loss = cross-entropy +
 *      0.1 * Huber(log step); then the stop labels are re-measured on traces
 *      of the search started from the predicted clusters' entry lists and
 *      training continues for the remaining epochs.
 * Afterwards option use_model = 1 makes svf_search start confident queries
 * from their cluster's list with a predicted expansion cap; others (softmax
 * below model_conf) run plain search.  n >= 1024; 2 <= n_clusters <= 256.
 * *last_loss (may be NULL) receives the mean loss of the last epoch. */
int svf_model_fit(svf_index *ix, const float *train_queries, int64_t n, int32_t k, int32_t beam,
                  int32_t n_clusters, int32_t epochs, float *last_loss);

/* Plain search (random entry points, no predictor, no cap) that also
 * reports, per query, the expansion count after which its k nearest last
 * changed: the stopping-step label that svf_model_fit trains on (step 2
 * above).  queries: nq x dim FP32, host; out_ids / out_dists: nq x k, host;
 * out_last_change: nq int32, host (0 when the first pool already held the
 * final k nearest).  Errors as svf_search; SVF_E_BUSY while serving. */
int svf_search_trace(svf_index *ix, const float *queries, int64_t nq, int32_t k, int32_t beam,
                     int32_t *out_ids, float *out_dists, int32_t *out_last_change);

/* The trained predictor as svf_search uses it (so that a replay of the
 * learned form can be checked outside the library): *n_clusters and
 * *entry_cap (may be NULL); params (may be NULL; params_cap floats, at least
 * the count svf_mlp_num_params gives for din = dim, hidden 256, n_clusters)
 * receives W1 b1 W2 b2 W3 b3 in svf_mlp's flat order with the weights on the
 * BF16 grid the forward pass multiplies by; entry_lists (may be NULL;
 * lists_cap ints, at least n_clusters x entry_cap) receives each cluster's
 * entry ids (-1 padded).  SVF_E_NOTFOUND before svf_model_fit; SVF_E_INVAL
 * for a short buffer.  Host memory, owned by the caller. */
int svf_model_get(const svf_index *ix, int32_t *n_clusters, int32_t *entry_cap, float *params,
                  int64_t params_cap, int32_t *entry_lists, int64_t lists_cap);

/* The predictor on its own (the network svf_model_fit trains), for checks of
 * its forward pass, gradients and training.  Parameters are one flat FP32
 * vector: W1 (din x hidden), b1, W2 (hidden x hidden), b2,
 * W3 (hidden x (n_clusters + 1)), b3, row-major (input x output).  Weights are
 * held on the BF16 grid (FP32 masters while training); activations are
 * rounded to BF16 between layers; products accumulate in FP32.  All pointers
 * are host memory. */
typedef struct svf_mlp svf_mlp;
int svf_mlp_create(int32_t din, int32_t hidden, int32_t n_clusters, uint64_t seed, svf_mlp **out);
int svf_mlp_destroy(svf_mlp *m);
int svf_mlp_num_params(const svf_mlp *m, int64_t *n);
int svf_mlp_set_params(svf_mlp *m, const float *params);
int svf_mlp_get_params(const svf_mlp *m, float *params);
/* out: n x (n_clusters + 1) outputs (cluster logits, then log stop step). */
int svf_mlp_forward(svf_mlp *m, const float *x, int64_t n, float *out);
/* Mean over n samples of cross-entropy(label) + lambda * Huber(z_last -
 * log_stop; delta); grad receives its gradient in the flat parameter order. */
int svf_mlp_loss_grad(svf_mlp *m, const float *x, const int32_t *label, const float *log_stop,
                      int64_t n, float lambda, float delta, float *loss, float *grad);
/* Adam (lr, betas 0.9 / 0.999) over `epochs` passes of consecutive batches. */
int svf_mlp_train(svf_mlp *m, const float *x, const int32_t *label, const float *log_stop,
                  int64_t n, int32_t epochs, int32_t batch, float lr, float lambda, float delta,
                  float *last_loss);
const char *svf_mlp_last_error(void);

/* Search whose pools start from caller-given entry points: entries is nq x
 * ecap ids (host memory, -1 = unused); every distinct alive id of a query's
 * list is evaluated and the best `beam` of them start its pool; a list with
 * no usable id falls back to random entry points.  max_iters (nq
 * ints, may be NULL) caps each query's expansions (0 = none).  This is the
 * search step of the learned form with the predictions supplied directly. */
int svf_search_listed(svf_index *ix, const float *queries, int64_t nq, int32_t k, int32_t beam,
                      const int32_t *entries, int32_t ecap, const int32_t *max_iters,
                      int32_t *out_ids, float *out_dists);

/* Serving loop (the paper's real-time coordination, Sec. 4.4, on one GPU).
 * A dispatcher thread owns the index between svf_serve_start and
 * svf_serve_stop; during that time the direct calls above return SVF_E_BUSY
 * (svf_stats_get and svf_get_option still work).
 *  - Search requests are coalesced in arrival order into batches of at most
 *    max_batch queries (same k and beam) and run on `streams` search streams
 *    (1..16), so batches overlap on the device.  A batch is admitted when a
 *    stream is free and its buffers fit in the HBM budget (hbm_budget bytes,
 *    0 = 80% of the free device memory at start); a request that can never
 *    fit fails with SVF_E_NOMEM.
 *  - Inserts and deletes apply one at a time in arrival order.  An insert's
 *    search and prune phases run while search batches continue; its commit
 *    and every delete wait for in-flight search batches.  Each committed
 *    insert batch (insert_batch_max vectors) or delete advances the epoch.
 *  - With consolidate_async, a consolidation runs beside all of this and is
 *    merged, between mutations and with no search in flight, once it has
 *    finished; the merge advances the epoch too.
 *  - A search sees the epoch committed when its batch launches, so its
 *    result equals that of the same search issued alone at that point.
 * Submit calls copy their inputs and return a ticket at once; output buffers
 * must stay valid until svf_wait returns for that ticket.  The learned form
 * (use_model) is not served. */
typedef struct svf_request_info {
    int32_t status;          /* SVF_OK or the request's error                 */
    double queue_ms;         /* submit -> launch on the device (host clock)   */
    double total_ms;         /* submit -> completion seen by the dispatcher    */
    int64_t batch_queries;   /* queries of the device batch a search ran in    */
    int64_t epoch;           /* epoch a search saw / a mutation produced        */
} svf_request_info;
int svf_serve_start(svf_index *ix, int32_t streams, int64_t max_batch, int64_t hbm_budget);
int svf_serve_stop(svf_index *ix);   /* finishes every submitted request first */
int svf_submit_search(svf_index *ix, const float *queries, int64_t nq, int32_t k, int32_t beam,
                      int32_t *out_ids, float *out_dists, uint64_t *ticket);
int svf_submit_insert(svf_index *ix, const float *vecs, int64_t n, int32_t *out_ids,
                      uint64_t *ticket);
int svf_submit_delete(svf_index *ix, const int32_t *ids, int64_t n, uint64_t *ticket);
/* Block until the request finishes (timeout_s < 0: no limit); info may be
 * NULL.  Returns the request's status; a ticket can be waited for once. */
int svf_wait(svf_index *ix, uint64_t ticket, double timeout_s, svf_request_info *info);

/* Statistics of the index and of its last calls. */
int svf_stats_get(const svf_index *ix, svf_stats *out);

/* Copy the graph out (host memory): rows (n_slots x degree ids), edge_d
 * (n_slots x degree FP32 distances) and alive (n_slots bytes), each may be
 * NULL.  cap_slots must be >= n_slots. */
int svf_export_graph(const svf_index *ix, int32_t *rows, float *edge_d, uint8_t *alive,
                     int64_t cap_slots);

/* The tiered store's cache (Sec. 4.2's mapping table, seen from the slots):
 * slot_ids receives, for each of the cache_slots slots, the id it holds or
 * -1 (host memory, cap >= cache_slots entries); *clock (may be NULL) the
 * position of Alg. 2's clock hand.  No tiered store: zero slots. */
int svf_cache_slots(const svf_index *ix, int32_t *slot_ids, int64_t cap, int64_t *clock);

/* Sec. 4.3's threshold from measured costs: theta = T_transfer / (T_miss -
 * T_hit), the access count from which promoting a vector pays for itself
 * (Eq. 1 with gain = 0).  Measured on this GPU with 65,536 random rows per
 * probe (median of five runs): T_hit, the per-row time of a distance over
 * rows read from the HBM cache; T_miss, the cost of a miss on the path in
 * force: with cache_cpu_miss the host cores' time per distance (the paper's
 * T_CPU, on the worker threads of the co-processed search), else the GPU's
 * time per distance over host rows read across the link; T_transfer, the
 * per-row time of copying 2048
 * host rows into HBM (one promotion batch).  Sets cache_theta (and the floor
 * of its adaptation) to theta; out (4 doubles, may be NULL) receives T_hit,
 * T_miss, T_transfer in ns per row, and theta.  Needs a tiered store that
 * holds at least one vector; SVF_E_INTERNAL if host reads measure no slower
 * than cached ones. */
int svf_cache_calibrate(svf_index *ix, double *out);

/* Replace the state of an EMPTY index by n vectors, their rows, edge
 * distances and alive flags (host memory).  Used to start two
 * implementations from one identical state. */
int svf_import_graph(svf_index *ix, const float *vecs, int64_t n, const int32_t *rows,
                     const float *edge_d, const uint8_t *alive);

/* Checkpoint to a file: the FP32 vectors, rows, edge distances, alive flags,
 * deletion counters and the options that shape results (seed, beam_insert,
 * entry_samples, max_iters, search_width, visited_slots, visited_compact,
 * repair_c, prune_cap, consolidate_frac, localized_repair, insert_batch_max,
 * precision, rerank).  Not saved: a fitted predictor, the tiered-store state and the
 * serving loop (a loaded index starts without them).  SVF_E_BUSY while a
 * background consolidation is pending.  Format: the 8 bytes
 * "SVFIDX01", a fixed header (format version 2; version 1 files, which lack
 * localized_repair, still load), the arrays, then a 64-bit checksum of all
 * that precedes it; little-endian.  Not while serving (SVF_E_BUSY); a file that
 * cannot be written gives SVF_E_INTERNAL and may be left incomplete. */
int svf_save(const svf_index *ix, const char *path);
/* Resume from svf_save's file into a new handle (*out; NULL on failure).
 * Missing file: SVF_E_NOTFOUND.  Wrong magic or version, truncation or a
 * checksum mismatch: SVF_E_INVAL.  Search results equal those of the index
 * that was saved. */
int svf_load(const char *path, svf_index **out);

/* Thread-local message of the last failing call on this thread. */
const char *svf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SVF_H */
