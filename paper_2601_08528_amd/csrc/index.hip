// C ABI of the library: index state in HBM, batch orchestration of the
// search, insertion and deletion kernels, option handling and errors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "index.hpp"
#include "index_internal.hpp"
#include "kernels.hpp"

using svf::DevBuf;

namespace svf_detail {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
int hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? SVF_E_NOMEM : SVF_E_DEVICE;
}

constexpr int kMaxBeam = 512;          // insertion pool (beam_insert)
constexpr int kMaxSearchBeam = 1024;   // search pool: 2 x 1024 keys of LDS per wave
constexpr int kMaxEntries = 1024;

int tier_release(svf_index* ix, const int32_t* ids, int64_t n);
// The device in-degree array while it is kept current, else null.
int32_t* kept_indegree(svf_index* ix) {
  return ix->tier.on && ix->tier.e_in_valid ? ix->tier.e_in_d.as<int32_t>() : nullptr;
}
int tier_admit(svf_index* ix, int64_t id0, int64_t n);
int tier_apply(svf_index* ix, const std::vector<int32_t>& place, hipStream_t st);
int bg_log(svf_index* ix, const int32_t* fwd, const float* fwd_d, int64_t b, hipStream_t st);
void bg_join(svf_index* ix);

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

int beam_insert(const svf_index* ix) {
  return ix->opt.beam_insert > 0 ? ix->opt.beam_insert : std::min(2 * ix->R, kMaxBeam);
}
// Candidates one wave prunes in LDS.  Longer lists go to the long-list
// kernels (no list is cut), unless prune_cap is set: then every list is cut
// to its prune_cap nearest candidates.  The LDS lists hold a top-up search
// pool beside fewer than R candidates (R - 1 + beam_insert).
int prune_cap(const svf_index* ix) {
  if (ix->opt.prune_cap > 0) return ix->opt.prune_cap;
  return std::max(4 * ix->R, ix->R + beam_insert(ix));
}
bool lists_uncut(const svf_index* ix) { return ix->opt.prune_cap == 0; }
// Candidates the one-wave reverse-edge prune holds in LDS when lists are not
// cut: most targets take R alive entries plus a few new neighbours, and the
// smaller pool leaves room for more waves per compute unit; longer lists go
// to the long-list kernels.
int reverse_lds_cap(const svf_index* ix) { return std::max(128, (ix->R + 64 + 63) / 64 * 64); }

// ---- candidate lists longer than the LDS kernels hold ------------------------------
constexpr int64_t kLongRoundKeys = (int64_t)1 << 24;   // raw keys per round of the long-list kernels

// Lay out the long-list workspace for n lists of raw lengths len[] (host) and
// point L at it; d_dst (device, n entries) names each list's output row.
int long_layout(svf::LongScratch& s, const int32_t* len, int n, const int32_t* d_dst, int skip_m,
                svf::LongLists* L, int64_t* hash_words, int64_t* cnt_words, int* max_len,
                hipStream_t st) {
  std::vector<int64_t> meta(3 * (size_t)n + 2);
  int64_t* off = meta.data();
  int64_t* hoff = off + n + 1;
  int64_t* coff = hoff + n + 1;
  off[0] = 0;
  hoff[0] = 0;
  int64_t c = 0;
  int mx = 0;
  for (int l = 0; l < n; ++l) {
    off[l + 1] = off[l] + len[l];
    int64_t S = 64;
    while (S < 2 * (int64_t)len[l]) S <<= 1;
    hoff[l + 1] = hoff[l] + 2 * S;
    coff[l] = c;
    c += 2 * (int64_t)len[l] + 1;
    mx = std::max(mx, len[l]);
  }
  int64_t* dmeta;
  uint64_t* keys;
  uint32_t *hash, *cnt;
  int32_t* m;
  int rc;
  if ((rc = scratch_grow(s.meta, meta.size(), &dmeta)) || (rc = scratch_grow(s.keys, (size_t)off[n], &keys)) ||
      (rc = scratch_grow(s.hash, (size_t)hoff[n], &hash)) || (rc = scratch_grow(s.cnt, (size_t)c, &cnt)) ||
      (rc = scratch_grow(s.m, (size_t)n, &m)))
    return rc;
  CK(hipMemcpyAsync(dmeta, meta.data(), meta.size() * 8, hipMemcpyHostToDevice, st));
  CK(hipStreamSynchronize(st));       // the host copy of the layout goes out of scope
  L->n = n;
  L->off = dmeta;
  L->hoff = dmeta + n + 1;
  L->coff = dmeta + 2 * (n + 1);
  L->dst = d_dst;
  L->keys = keys;
  L->m = m;
  L->hash = hash;
  L->cnt = cnt;
  L->skip_m = skip_m;
  *hash_words = hoff[n];
  *cnt_words = c;
  *max_len = mx;
  return SVF_OK;
}

// Split n lists of raw lengths len[] into consecutive rounds of at most
// kLongRoundKeys raw keys; calls run(l0, l1) per round.
template <class F>
int long_rounds(const std::vector<int32_t>& len, F run) {
  const int n = (int)len.size();
  for (int l0 = 0; l0 < n;) {
    int l1 = l0;
    int64_t tot = 0;
    while (l1 < n && (l1 == l0 || tot + len[l1] <= kLongRoundKeys)) tot += len[l1++];
    int rc = run(l0, l1);
    if (rc) return rc;
    l0 = l1;
  }
  return SVF_OK;
}

// Reverse-edge prune of the n_targets staged targets: the LDS kernel for
// every target, then the long-list kernels rewrite the targets whose alive
// row entries plus incoming keys exceed its capacity.
int reverse_prune_all(svf_index* ix, svf::ReverseArgs& ra, int n_targets, hipStream_t st) {
  if (n_targets <= 0) return SVF_OK;
  if (!lists_uncut(ix)) {
    CK(svf::launch_reverse_prune(ra, n_targets, st));
    return SVF_OK;
  }
  svf::LongScratch& s = ix->lrev;
  int32_t* q;
  int rc;
  if ((rc = scratch_grow(s.q, 2 * (size_t)n_targets + 1, &q))) return rc;
  int32_t *qk = q, *qlen = q + n_targets, *nq = q + 2 * n_targets;
  CK(svf::launch_fill_u32(nq, 1, 0u, st));
  svf::ReverseArgs rq = ra;
  rq.cap = reverse_lds_cap(ix);
  rq.long_q = qk;
  rq.long_len = qlen;
  rq.long_n = nq;
  CK(svf::launch_reverse_prune(rq, n_targets, st));
  int32_t n_long = 0;
  CK(hipMemcpyAsync(&n_long, nq, 4, hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  if (n_long == 0) return SVF_OK;
  s.lists += n_long;
  std::vector<int32_t> len(n_long);
  CK(hipMemcpyAsync(len.data(), qlen, (size_t)n_long * 4, hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  for (int32_t x : len)
    if (x > svf::kLongMaxKeys)
      return fail(SVF_E_INVAL, "a vertex would take more than 16384 reverse-edge candidates from one "
                               "insert batch: use smaller batches (insert_batch_max)");
  svf::LongRows rows{ra.graph, ra.fwd_ids, ra.rows_below ? ra.rows_below : ra.n0, ra.R};
  return long_rounds(len, [&](int l0, int l1) {
    svf::LongLists L{};
    int64_t hw, cw;
    int mx;
    int rc2 = long_layout(s, len.data() + l0, l1 - l0, qk + l0, 0, &L, &hw, &cw, &mx, st);
    if (rc2) return rc2;
    CK(svf::launch_reverse_gather(ra, qk + l0, L, st));
    CK(svf::launch_long_sort(L, mx, st));
    CK(svf::launch_long_prune(L, rows, ra.trow, ra.trow_d, hw, cw, st));
    return (int)SVF_OK;
  });
}
// Reduced-precision traversal store: FP16/BF16 rows of `stride` 2-byte
// elements; FP8 rows of round_up(dim, 16) codes followed, after all cap rows,
// by cap FP32 scales.
int64_t lp_stride(const svf_index* ix, int prec) {
  return prec == 3 ? round_up(ix->dim, 16) : ix->stride;
}
size_t lp_row_bytes(const svf_index* ix, int prec) {
  return prec == 3 ? (size_t)lp_stride(ix, 3) : (size_t)ix->stride * 2;
}
size_t lp_bytes(const svf_index* ix, int prec, int64_t cap) {
  return (size_t)cap * lp_row_bytes(ix, prec) + (prec == 3 ? (size_t)cap * 4 : 0);
}
float* lp_scale(void* veclp, const svf_index* ix, int prec, int64_t cap) {
  if (prec != 3 || !veclp) return nullptr;
  return reinterpret_cast<float*>(static_cast<char*>(veclp) + (size_t)cap * lp_row_bytes(ix, prec));
}

// Visited-table slots of one search.  0 (the default) picks by traversal
// precision: 4096 for FP32 and 2048 for reduced precision, whose cheaper
// distances gain more from the smaller table's higher LDS occupancy than they
// lose to its extra re-evaluations, as long as the ids fit its 16-bit tags
// (2^24 ids at 2048 slots); beyond that 4096.  The size never changes results.
int visited_slots(const svf_index* ix, int E) {
  int T = ix->opt.visited_slots;
  if (T == 0) T = (ix->veclp_prec != 0 && ix->n_slots <= (int64_t)1 << 24) ? 2048 : 4096;
  while (T < 2 * E) T <<= 1;   // entry phase needs an exact table
  return T;
}


// Grow the device arrays to hold `need` id slots, keeping the contents.
// One pinned host allocation is kept below this size: larger ones have failed
// well below what pinned memory holds in all.
constexpr int64_t kHostSegBytes = int64_t(4) << 30;

// Rows per host segment, as a power of two: the host_segment_rows option, or
// the most rows whose segment stays within kHostSegBytes (at least 4096).
int host_seg_shift(const svf_index* ix) {
  int s = 10;
  if (ix->tier.seg_rows_opt > 0) {
    while ((int64_t(1) << s) < ix->tier.seg_rows_opt) ++s;
    return s;
  }
  s = 12;
  while ((int64_t(2) << s) * ix->stride * 4 <= kHostSegBytes) ++s;
  return s;
}

// Make the tiered store's host segments hold rows [0, cap).  Rows already
// stored stay where they are, except in a last segment that grows (its rows
// are copied into the larger allocation); new rows are zero.  On failure the
// store keeps its previous rows and capacity.
int tier_grow_host(svf_index* ix, int64_t cap) {
  svf::TierState& T = ix->tier;
  const int64_t S = int64_t(1) << T.seg_shift;
  const int64_t rb = ix->stride * 4;
  const int64_t nseg = (cap + S - 1) / S;
  for (int64_t i = 0; i < nseg; ++i) {
    const int64_t want = (i + 1 < nseg) ? S : cap - i * S;
    const int64_t have = i < (int64_t)T.seg.size() ? T.seg_alloc[i] : 0;
    if (have >= want) continue;
    float* p = nullptr;
    const hipError_t e = hipHostMalloc((void**)&p, (size_t)(want * rb), 0);
    if (e != hipSuccess) {
      int64_t held = 0;
      for (int64_t r : T.seg_alloc) held += r * rb;
      char what[160];
      std::snprintf(what, sizeof what,
                    "pinned host segment of the tiered store (%.2f GiB already pinned in %zu "
                    "segments of at most %.2f GiB)",
                    (double)held / (1 << 30), T.seg.size(), (double)(S * rb) / (1 << 30));
      return hip_fail(e, what);
    }
    if (have > 0) std::memcpy(p, T.seg[i], (size_t)(have * rb));
    std::memset(reinterpret_cast<char*>(p) + have * rb, 0, (size_t)((want - have) * rb));
    if (i < (int64_t)T.seg.size()) {
      (void)hipHostFree(T.seg[i]);
      T.seg[i] = p;
      T.seg_alloc[i] = want;
    } else {
      T.seg.push_back(p);
      T.seg_alloc.push_back(want);
    }
  }
  CK(T.seg_d.ensure(T.seg.size() * sizeof(float*)));
  CK(hipMemcpy(T.seg_d.p, T.seg.data(), T.seg.size() * sizeof(float*), hipMemcpyHostToDevice));
  return SVF_OK;
}

int row_scales_sync(svf_index* ix, hipStream_t st);

int reserve(svf_index* ix, int64_t need) {
  if (need <= ix->cap) return SVF_OK;
  bg_join(ix);                              // it reads the vector stores that move below
  if (need > (int64_t)INT32_MAX - 64) return fail(SVF_E_INVAL, "index would exceed int32 ids");
  int64_t cap = std::max<int64_t>({need, ix->cap * 2, 1024});
  cap = round_up(cap, 64);
  const int64_t words = cap / 32;
  float *v32 = nullptr, *ed = nullptr;
  void* vlp = nullptr;
  int32_t *g = nullptr, *tc = nullptr, *ti = nullptr;
  uint32_t* al = nullptr;
  auto cleanup = [&]() {
    if (v32) (void)hipFree(v32);
    if (vlp) (void)hipFree(vlp);
    if (g) (void)hipFree(g);
    if (ed) (void)hipFree(ed);
    if (al) (void)hipFree(al);
    if (tc) (void)hipFree(tc);
    if (ti) (void)hipFree(ti);
  };
  hipError_t e = hipSuccess;
  const bool tier = ix->tier.on;
  int32_t* tmap = nullptr;
  if (tier) {
    // the host store grows by segments in place (rows already stored stay put)
    const int rc = tier_grow_host(ix, cap);
    if (rc) return rc;
    if ((e = hipMalloc(&tmap, cap * 4)) != hipSuccess) return hip_fail(e, "index allocation");
  }
  if ((!tier && (e = hipMalloc(&v32, cap * ix->stride * 4)) != hipSuccess) ||
      (ix->veclp_prec && (e = hipMalloc(&vlp, lp_bytes(ix, ix->veclp_prec, cap))) != hipSuccess) ||
      (e = hipMalloc(&g, cap * ix->R * 4)) != hipSuccess ||
      (e = hipMalloc(&ed, cap * ix->R * 4)) != hipSuccess ||
      (e = hipMalloc(&al, words * 4)) != hipSuccess ||
      (e = hipMalloc(&tc, cap * 4)) != hipSuccess || (e = hipMalloc(&ti, cap * 4)) != hipSuccess) {
    cleanup();
    if (tmap) (void)hipFree(tmap);
    return hip_fail(e, "index allocation");
  }
  hipStream_t st = ix->stream;
  const int64_t n = ix->n_slots;
  ix->tier.e_in_valid = false;             // sized by capacity: counted again when next needed
  if (tier) {
    CK(svf::launch_fill_u32(tmap, cap, 0xffffffffu, st));
    if (n > 0 && ix->tier.map) CK(hipMemcpyAsync(tmap, ix->tier.map, n * 4, hipMemcpyDeviceToDevice, st));
    ix->tier.where.resize(cap, -1);
    ix->tier.fr.resize(cap);
    ix->tier.freq.resize(cap, 0);
    ix->tier.last.resize(cap, -1);
  } else {
    CK(svf::launch_fill_u32(v32, cap * ix->stride, 0u, st));
  }
  if (vlp) CK(svf::launch_fill_u32(vlp, lp_bytes(ix, ix->veclp_prec, cap) / 4, 0u, st));
  CK(svf::launch_fill_u32(g, cap * ix->R, 0xffffffffu, st));
  CK(svf::launch_fill_u32(ed, cap * ix->R, 0x7f800000u, st));
  CK(svf::launch_fill_u32(al, words, 0u, st));
  CK(svf::launch_fill_u32(tc, cap, 0u, st));
  if (n > 0) {
    if (!tier) CK(hipMemcpyAsync(v32, ix->vec32, n * ix->stride * 4, hipMemcpyDeviceToDevice, st));
    if (vlp) {
      const int p = ix->veclp_prec;
      CK(hipMemcpyAsync(vlp, ix->veclp, n * lp_row_bytes(ix, p), hipMemcpyDeviceToDevice, st));
      if (p == 3)
        CK(hipMemcpyAsync(lp_scale(vlp, ix, p, cap), lp_scale(ix->veclp, ix, p, ix->cap), n * 4,
                          hipMemcpyDeviceToDevice, st));
    }
    CK(hipMemcpyAsync(g, ix->graph, n * ix->R * 4, hipMemcpyDeviceToDevice, st));
    CK(hipMemcpyAsync(ed, ix->edge_d, n * ix->R * 4, hipMemcpyDeviceToDevice, st));
    CK(hipMemcpyAsync(al, ix->alive, ((n + 31) / 32) * 4, hipMemcpyDeviceToDevice, st));
  }
  CK(hipStreamSynchronize(st));
  if (tier) {
    if (ix->tier.map) (void)hipFree(ix->tier.map);
    ix->tier.map = tmap;
  } else {
    if (ix->vec32) (void)hipFree(ix->vec32);
    ix->vec32 = v32;
  }
  if (ix->veclp) (void)hipFree(ix->veclp);
  if (ix->graph) (void)hipFree(ix->graph);
  if (ix->edge_d) (void)hipFree(ix->edge_d);
  if (ix->alive) (void)hipFree(ix->alive);
  ix->veclp = vlp;
  ix->graph = g;
  ix->edge_d = ed;
  ix->alive = al;
  ix->cap = cap;
  // tcount / tidx are per-slot scratch of the reverse-edge step
  static_assert(sizeof(int32_t) == 4, "");
  ix->s_misc[10].release();
  ix->s_misc[11].release();
  ix->s_misc[10].p = tc; ix->s_misc[10].bytes = cap * 4;
  ix->s_misc[11].p = ti; ix->s_misc[11].bytes = cap * 4;
  const int rc = row_scales_sync(ix, st);     // sized by capacity: filled again
  if (rc) return rc;
  CK(hipStreamSynchronize(st));
  return SVF_OK;
}

int32_t* tcount(svf_index* ix) { return ix->s_misc[10].as<int32_t>(); }
int32_t* tidx(svf_index* ix) { return ix->s_misc[11].as<int32_t>(); }

int store_lowp_rows(svf_index* ix, int64_t row0, int64_t n, hipStream_t st);

// FP8 traversal keeps each row's vector scales beside it (nscale) when asked,
// or by size once the per-vector scales (4 B each) are past what the caches
// hold: then a scale read costs a cache line per distance.
bool row_scales_wanted(const svf_index* ix) {
  if (ix->veclp_prec != 3 || ix->cap == 0) return false;
  if (ix->opt.fp8_row_scales >= 0) return ix->opt.fp8_row_scales == 1;
  return ix->cap >= (int64_t(1) << 24);
}

// Allocate (capacity rows) and fill, or free, the row scales to match
// row_scales_wanted.
int row_scales_sync(svf_index* ix, hipStream_t st) {
  if (ix->nscale) (void)hipFree(ix->nscale);
  ix->nscale = nullptr;
  if (!row_scales_wanted(ix)) return SVF_OK;
  CK(hipMalloc(&ix->nscale, (size_t)ix->cap * ix->R * 4));
  CK(svf::launch_row_scales(ix->graph, ix->R, nullptr, 0, ix->n_slots,
                            lp_scale(ix->veclp, ix, 3, ix->cap), ix->nscale, st));
  return SVF_OK;
}

// Row scales of rows just written: the n rows of list, or rows [lo, lo + n).
int row_scales_rows(svf_index* ix, const int32_t* list, int64_t lo, int64_t n, hipStream_t st) {
  if (!ix->nscale || n <= 0) return SVF_OK;
  CK(svf::launch_row_scales(ix->graph, ix->R, list, lo, n, lp_scale(ix->veclp, ix, 3, ix->cap),
                            ix->nscale, st));
  return SVF_OK;
}

// Make the reduced-precision copy match the chosen precision.
int sync_lowp(svf_index* ix) {
  const int prec = ix->opt.precision;
  if (prec == ix->veclp_prec) return row_scales_wanted(ix) == (ix->nscale != nullptr)
                                        ? SVF_OK : row_scales_sync(ix, ix->stream);
  bg_join(ix);                              // it may be reading the store freed below
  if (ix->veclp) (void)hipFree(ix->veclp);
  ix->veclp = nullptr;
  ix->veclp_prec = prec;
  if (prec == 0 || ix->cap == 0) return row_scales_sync(ix, ix->stream);
  CK(hipMalloc(&ix->veclp, lp_bytes(ix, prec, ix->cap)));
  CK(svf::launch_fill_u32(ix->veclp, lp_bytes(ix, prec, ix->cap) / 4, 0u, ix->stream));
  int rc = store_lowp_rows(ix, 0, ix->n_slots, ix->stream);
  if (rc || (rc = row_scales_sync(ix, ix->stream))) return rc;
  CK(hipStreamSynchronize(ix->stream));
  return SVF_OK;
}

// Calls f(row0, nrows, src) for the runs of rows [at, at + n) that are
// contiguous in the FP32 store (one run in HBM, one per segment when tiered);
// src is the address of row row0.
template <class F>
int for_store_runs(svf_index* ix, int64_t at, int64_t n, F&& f) {
  while (n > 0) {
    int64_t len = n;
    float* src = nullptr;
    if (ix->tier.on) {
      const int64_t S = int64_t(1) << ix->tier.seg_shift;
      len = std::min<int64_t>(n, S - (at & (S - 1)));
      src = ix->tier.hrow(at, ix->stride);
    } else {
      src = ix->vec32 + at * ix->stride;
    }
    const int rc = f(at, len, src);
    if (rc) return rc;
    at += len;
    n -= len;
  }
  return SVF_OK;
}

// Reduced-precision rows [row0, row0 + n) from the FP32 store.
int store_lowp_rows(svf_index* ix, int64_t row0, int64_t n, hipStream_t st) {
  const int p = ix->veclp_prec;
  if (!p || n <= 0) return SVF_OK;
  return for_store_runs(ix, row0, n, [&](int64_t r0, int64_t len, float* src) -> int {
    CK(svf::launch_store_lowp(src, ix->stride, ix->dim, ix->veclp, lp_stride(ix, p),
                              lp_scale(ix->veclp, ix, p, ix->cap), r0, len, p, st));
    return SVF_OK;
  });
}

// Copy n rows (pitch dim floats, device memory) into slots [at, at + n).
int store_rows(svf_index* ix, const float* d_src, int64_t n, int64_t at, hipStream_t st) {
  if (n <= 0) return SVF_OK;
  const int rc = for_store_runs(ix, at, n, [&](int64_t r0, int64_t len, float* dst) -> int {
    CK(hipMemcpy2DAsync(dst, ix->stride * 4, d_src + (r0 - at) * ix->dim, ix->dim * 4,
                        ix->dim * 4, len, hipMemcpyDefault, st));
    return SVF_OK;
  });
  if (rc) return rc;
  return store_lowp_rows(ix, at, n, st);
}

const void* traversal_store(const svf_index* ix) {
  return ix->veclp_prec ? ix->veclp : (const void*)ix->vec32;
}

svf::SearchArgs base_args(const svf_index* ix) {
  svf::SearchArgs a{};
  a.vec = traversal_store(ix);
  a.vec32 = ix->vec32;
  a.stride = ix->stride;
  a.vstride = ix->veclp_prec ? lp_stride(ix, ix->veclp_prec) : ix->stride;
  a.vscale = lp_scale(ix->veclp, ix, ix->veclp_prec, ix->cap);
  a.nscale = ix->veclp_prec == 3 ? ix->nscale : nullptr;
  a.dim = ix->dim;
  a.graph = ix->graph;
  a.R = ix->R;
  a.alive = ix->alive;
  a.n_slots = (int32_t)ix->n_slots;
  a.n_alive = (int32_t)ix->n_alive;
  a.metric = ix->metric;
  a.max_iters = ix->opt.max_iters;
  if (ix->tier.on) {
    a.hsegs = ix->tier.segs();
    a.tmap = ix->tier.map;
    a.tcache = ix->tier.cache;
  }
  return a;
}

void set_beam(svf::SearchArgs& a, const svf_index* ix, int L) {
  a.L = L;
  int Lp = 64;
  while (Lp < L) Lp <<= 1;
  a.L_pow2 = Lp;
  a.E = ix->opt.entry_samples > 0 ? ix->opt.entry_samples : L;
  a.T = visited_slots(ix, a.E);
  a.rerank = (ix->veclp_prec != 0 && ix->opt.rerank) ? 1 : 0;
  a.vis_compact = ix->opt.visited_compact;
  a.width = ix->opt.search_width;
  a.coop_max_nq = ix->opt.coop_max_batch;
}

// Milliseconds between two recorded events, 0 when they cannot be timed.  A
// failure here must not stay behind as the thread's last HIP error, where
// the next launch check would report it.
float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess) {
    (void)hipGetLastError();
    return 0.f;
  }
  return ms;
}

// Insertion of one batch, in two parts.  insert_prepare stores the vectors in
// slots beyond n_slots and runs the batched search, the forward prune and the
// reverse-edge grouping and prune into staged rows: it only reads state that
// searches also read, so searches may run beside it.  insert_commit writes
// the staged rows, the new rows and the alive bits and advances n_slots.
int insert_prepare(svf_index* ix, const float* d_vecs, int64_t b, PendingInsert* p) {
  p->b = b;
  p->n0 = ix->n_slots;
  p->seed = ix->n_slots == 0;
  p->n_targets = 0;
  if (b <= 0) return SVF_OK;
  int rc = reserve(ix, ix->n_slots + b);
  if (rc) return rc;
  hipStream_t st = ix->stream;
  const int R = ix->R;
  const int64_t n0 = ix->n_slots;
  if (p->seed) {
    // empty index: the seed rule (exact R-nearest among the seed vectors)
    if (b > 4 * R) return fail(SVF_E_INTERNAL, "seed batch larger than 4 * degree");
    rc = store_rows(ix, d_vecs, b, 0, st);
    if (rc) return rc;
    // the seed rows sit in the first host segment when tiered (it holds at
    // least 1024 rows)
    const float* v0 = ix->tier.on ? ix->tier.seg[0] : ix->vec32;
    CK(svf::launch_seed(v0, ix->stride, ix->dim, ix->metric, (int)b, R, ix->graph, ix->edge_d, st));
    CK(hipStreamSynchronize(st));
    return SVF_OK;
  }
  const int Lins = beam_insert(ix);
  rc = store_rows(ix, d_vecs, b, n0, st);
  if (rc) return rc;
  uint64_t *qkey, *pool;
  int32_t *fwd, *cnt;
  float* fwd_d;
  if ((rc = scratch(ix->s_qkey, b, &qkey)) || (rc = scratch(ix->s_pool, b * Lins, &pool)) ||
      (rc = scratch(ix->s_misc[0], b * R, &fwd)) || (rc = scratch(ix->s_misc[1], b * R, &fwd_d)) ||
      (rc = scratch(ix->s_misc[2], 8, &cnt)))
    return rc;
  // phase 1: batched search of the pre-batch graph
  CK(hipEventRecord(ix->ev0, st));
  svf::SearchArgs a = base_args(ix);
  set_beam(a, ix, Lins);
  a.max_iters = 0;
  a.k = 0;
  if (ix->tier.on) {
    // the batch's rows, read from HBM rather than across the host link
    float* qrows;
    if ((rc = scratch(ix->s_rows, (size_t)b * ix->stride, &qrows))) return rc;
    CK(hipMemcpy2DAsync(qrows, ix->stride * 4, d_vecs, ix->dim * 4, ix->dim * 4, b,
                        hipMemcpyDefault, st));
    a.queries = qrows;
  } else {
    a.queries = ix->vec32 + n0 * ix->stride;
  }
  a.qstride = ix->stride;
  a.nq = (int)b;
  a.out_pool = pool;
  a.n_slots = (int32_t)n0;
  CK(svf::launch_query_keys(a.queries, a.qstride, nullptr, ix->dim, a.nq, ix->opt.seed, qkey, st));
  a.qkey = qkey;
  CK(svf::launch_search(a, ix->veclp_prec, st));
  CK(hipEventRecord(ix->ev1, st));
  ix->st.ins_search_ms = elapsed(ix->ev0, ix->ev1);
  // phase 2: rank-based reordering of each candidate list -> forward rows
  CK(hipEventRecord(ix->ev0, st));
  svf::PruneArgs pa{};
  pa.cand = pool;
  pa.cstride = Lins;
  pa.cap = Lins;                  // the whole insertion pool (prune_cap cuts only update lists)
  pa.graph = ix->graph;
  pa.fwd = nullptr;
  pa.n_old = (int32_t)n0;
  pa.R = R;
  pa.out_ids = fwd;
  pa.out_d = fwd_d;
  pa.nlists = (int)b;
  CK(svf::launch_prune_lists(pa, st));
  CK(hipEventRecord(ix->ev1, st));
  ix->st.ins_prune_ms = elapsed(ix->ev0, ix->ev1);
  // phase 3: reverse edges grouped by target, re-pruned into staged rows
  CK(hipEventRecord(ix->ev0, st));
  svf::ReverseArgs& ra = p->ra;
  ra = svf::ReverseArgs{};
  ra.fwd_ids = fwd;
  ra.fwd_d = fwd_d;
  ra.b = (int)b;
  ra.R = R;
  ra.n0 = (int32_t)n0;
  ra.tcount = tcount(ix);
  ra.tidx = tidx(ix);
  ra.graph = ix->graph;
  ra.edge_d = ix->edge_d;
  ra.alive = ix->alive;
  ra.cap = prune_cap(ix);
  const int64_t npairs = b * R;
  if ((rc = scratch(ix->s_misc[3], npairs, &ra.tlist))) return rc;
  ra.n_targets = cnt;
  CK(svf::launch_fill_u32(cnt, 1, 0u, st));
  CK(svf::launch_reverse_count(ra, st));
  int32_t n_targets = 0;
  CK(hipMemcpyAsync(&n_targets, cnt, 4, hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  const size_t nt = (size_t)n_targets;
  if ((rc = scratch_grow(ix->s_misc[4], nt + 1, &ra.off)) ||
      (rc = scratch_grow(ix->s_misc[5], nt + 2 + nt / 1024 + 2, &ra.cursor)) ||
      (rc = scratch(ix->s_misc[6], npairs, &ra.inc)) ||
      (rc = scratch_grow(ix->s_misc[7], nt * R, &ra.trow)) ||
      (rc = scratch_grow(ix->s_misc[8], nt * R, &ra.trow_d)))
    return rc;
  CK(svf::launch_reverse_scan_scatter(ra, n_targets, st));
  if ((rc = reverse_prune_all(ix, ra, n_targets, st))) return rc;
  CK(hipEventRecord(ix->ev1, st));
  ix->st.ins_reverse_ms = elapsed(ix->ev0, ix->ev1);
  p->n_targets = n_targets;
  return SVF_OK;
}

int insert_commit(svf_index* ix, PendingInsert* p) {
  if (p->b <= 0) return SVF_OK;
  hipStream_t st = ix->stream;
  if (p->seed) {
    ix->tier.e_in_valid = false;
    CK(svf::launch_set_alive(ix->alive, 0, p->b, st));
    const int rc = row_scales_rows(ix, nullptr, 0, p->b, st);
    if (rc) return rc;
    CK(hipStreamSynchronize(st));
    ix->n_slots = p->b;
    ix->n_alive = p->b;
    ++ix->graph_epoch;
    return tier_admit(ix, 0, p->b);
  }
  if (ix->bg.active) {
    if (p->n0 != ix->bg.n0 + ix->bg.log_n) return fail(SVF_E_INTERNAL, "insertion log out of order");
    int rc = bg_log(ix, p->ra.fwd_ids, p->ra.fwd_d, p->b, st);
    if (rc) return rc;
  }
  CK(hipEventRecord(ix->ev0, st));
  if (int32_t* e = kept_indegree(ix)) {
    CK(svf::launch_indegree_rows_delta(ix->graph, p->ra.tlist, p->n_targets, p->ra.trow, ix->R, e, st));
    CK(svf::launch_indegree_add(p->ra.fwd_ids, p->b * ix->R, e, st));
  }
  CK(svf::launch_commit_batch(p->ra, p->n_targets, ix->graph, ix->edge_d, ix->alive, st));
  int rc = row_scales_rows(ix, p->ra.tlist, 0, p->n_targets, st);
  if (rc || (rc = row_scales_rows(ix, nullptr, p->n0, p->b, st))) return rc;
  CK(hipEventRecord(ix->ev1, st));
  CK(hipStreamSynchronize(st));
  ix->st.ins_commit_ms = elapsed(ix->ev0, ix->ev1);
  ++ix->graph_epoch;
  ix->n_slots = p->n0 + p->b;
  ix->n_alive += p->b;
  return tier_admit(ix, p->n0, p->b);
}

// One insertion batch of b vectors already on the device (pitch dim).
int insert_batch(svf_index* ix, const float* d_vecs, int64_t b, int32_t* d_out_ids,
                 int32_t* h_out_ids) {
  if (b <= 0) return SVF_OK;
  PendingInsert p;
  int rc = insert_prepare(ix, d_vecs, b, &p);
  if (rc) return rc;
  rc = insert_commit(ix, &p);
  if (rc) return rc;
  const int64_t n0 = p.n0;
  if (h_out_ids)
    for (int64_t i = 0; i < b; ++i) h_out_ids[i] = (int32_t)(n0 + i);
  if (d_out_ids) {
    std::vector<int32_t> ids(b);
    for (int64_t i = 0; i < b; ++i) ids[i] = (int32_t)(n0 + i);
    CK(hipMemcpy(d_out_ids, ids.data(), b * 4, hipMemcpyHostToDevice));
  }
  return SVF_OK;
}

// What a repair / consolidation pass reads: the rows, edge distances and
// alive bits (the live graph, or a snapshot of it), the vectors, and the
// search used to top up short candidate lists (set up on the same graph).
struct RepairJob {
  const int32_t* graph;
  const float* edge_d;
  const uint32_t* alive;
  int64_t n_slots;
  const float* vec32;
  svf::HostSegs hsegs;        // tiered store: the FP32 rows (vec32 unused)
  int64_t stride;
  int dim, metric, R, cap, c_local, Lins, prec;
  bool uncut;                 // lists longer than cap go to the long-list kernels
  uint64_t seed;
  svf::SearchArgs proto;
};

RepairJob repair_job(svf_index* ix) {
  RepairJob j;
  j.graph = ix->graph;
  j.edge_d = ix->edge_d;
  j.alive = ix->alive;
  j.n_slots = ix->n_slots;
  j.vec32 = ix->vec32;
  j.hsegs = ix->tier.on ? ix->tier.segs() : svf::HostSegs{nullptr, 0};
  j.stride = ix->stride;
  j.dim = ix->dim;
  j.metric = ix->metric;
  j.R = ix->R;
  j.cap = prune_cap(ix);
  j.uncut = lists_uncut(ix);
  j.c_local = ix->opt.repair_c;
  j.Lins = beam_insert(ix);
  j.prec = ix->veclp_prec;
  j.seed = ix->opt.seed;
  j.proto = base_args(ix);
  set_beam(j.proto, ix, j.Lins);
  j.proto.max_iters = 0;
  j.proto.k = 0;
  return j;
}

// Repair (consolidate = 0) or consolidation (1) of the rows that name deleted
// ids: the new rows of the *n_aff affected vertices are left in s.list /
// s.rows / s.rows_d; nothing is committed.
int repair_compute(const RepairJob& j, int consolidate, svf::RepairScratch& s, hipStream_t st,
                   int32_t* n_aff_out) {
  const int R = j.R;
  const int cap = j.cap;
  int32_t *list, *cnt;
  int rc;
  *n_aff_out = 0;
  if ((rc = scratch_grow(s.list, std::max<int64_t>(j.n_slots, 1), &list)) || (rc = scratch_grow(s.cnt, 8, &cnt)))
    return rc;
  svf::RepairArgs a{};
  a.vec32 = j.vec32;
  a.hsegs = j.hsegs;
  a.stride = j.stride;
  a.dim = j.dim;
  a.metric = j.metric;
  a.R = R;
  a.graph = j.graph;
  a.edge_d = j.edge_d;
  a.alive = j.alive;
  a.n_slots = (int32_t)j.n_slots;
  a.consolidate = consolidate;
  a.c = consolidate ? R : j.c_local;
  a.cap = cap;
  a.list = list;
  a.n_list = cnt;
  a.n_topup = cnt + 1;
  CK(svf::launch_fill_u32(cnt, 2, 0u, st));
  CK(svf::launch_affected(a, st));
  int32_t n_aff = 0;
  CK(hipMemcpyAsync(&n_aff, cnt, 4, hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  if (n_aff == 0) return SVF_OK;
  int32_t *rows, *mcount, *topup, *topup_v, *over;
  float* rows_d;
  uint64_t* cand;
  const int64_t chunk = std::min<int64_t>(n_aff, 131072);
  if ((rc = scratch_grow(s.rows, (size_t)n_aff * R, &rows)) ||
      (rc = scratch_grow(s.rows_d, (size_t)n_aff * R, &rows_d)) ||
      (rc = scratch_grow(s.cand, (size_t)chunk * cap, &cand)) ||
      (rc = scratch_grow(s.mcount, chunk, &mcount)) || (rc = scratch_grow(s.topup, chunk, &topup)) ||
      (rc = scratch_grow(s.topup_v, chunk, &topup_v)) || (rc = scratch_grow(s.lg.q, 2 * (size_t)chunk, &over)))
    return rc;
  a.cand = cand;
  a.mcount = mcount;
  a.topup = topup;
  a.topup_v = topup_v;
  a.over_li = j.uncut ? over : nullptr;
  a.over_len = over + chunk;
  a.n_over = cnt + 2;
  const svf::LongRows lrows{j.graph, nullptr, (int32_t)j.n_slots, R};
  for (int64_t first = 0; first < n_aff; first += chunk) {
    const int count = (int)std::min<int64_t>(chunk, n_aff - first);
    CK(svf::launch_fill_u32(cnt + 1, 2, 0u, st));
    CK(svf::launch_repair_candidates(a, (int)first, count, st));
    int32_t hc[2] = {0, 0};
    CK(hipMemcpyAsync(hc, cnt + 1, 8, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    int32_t ntop = hc[0];
    const int32_t n_over = hc[1];
    if (n_over > 0) {
      // lists that offered more keys than the LDS walk kept: the same walk
      // again into the long-list staging area, sorted with repeats removed;
      // those of at most cap candidates go back to the LDS prune (and the
      // top-up when short), the others are pruned by the long-list kernels
      s.lg.lists += n_over;
      std::vector<int32_t> len(n_over);
      CK(hipMemcpyAsync(len.data(), a.over_len, (size_t)n_over * 4, hipMemcpyDeviceToHost, st));
      CK(hipStreamSynchronize(st));
      for (int32_t x : len)
        if (x > svf::kLongMaxKeys) return fail(SVF_E_INTERNAL, "repair candidate list above 16384");
      rc = long_rounds(len, [&](int l0, int l1) {
        svf::LongLists L{};
        int64_t hw, cw;
        int mx;
        int rc2 = long_layout(s.lg, len.data() + l0, l1 - l0, a.over_li + l0, cap, &L, &hw, &cw, &mx, st);
        if (rc2) return rc2;
        svf::RepairArgs ar = a;
        ar.over_li = a.over_li + l0;
        CK(svf::launch_repair_raw(ar, (int)first, L, st));
        CK(svf::launch_long_sort(L, mx, st));
        CK(svf::launch_repair_back(ar, (int)first, L, st));
        CK(svf::launch_long_prune(L, lrows, rows + first * R, rows_d + first * R, hw, cw, st));
        return (int)SVF_OK;
      });
      if (rc) return rc;
      CK(hipMemcpyAsync(&ntop, cnt + 1, 4, hipMemcpyDeviceToHost, st));
      CK(hipStreamSynchronize(st));
    }
    if (ntop > 0) {
      uint64_t *qkey, *pool;
      if ((rc = scratch_grow(s.qkey, ntop, &qkey)) || (rc = scratch_grow(s.pool, (size_t)ntop * j.Lins, &pool)))
        return rc;
      svf::SearchArgs q = j.proto;
      q.queries = j.vec32;
      q.qstride = j.stride;
      q.qids = topup_v;
      if (j.hsegs.seg) {
        // tiered: the vertices' own rows are staged in HBM first
        float* qrows;
        if ((rc = scratch_grow(s.qrows, (size_t)ntop * j.stride, &qrows))) return rc;
        CK(svf::launch_gather_rows(j.hsegs, topup_v, ntop, j.stride, qrows, st));
        q.queries = qrows;
        q.qids = nullptr;
      }
      q.nq = ntop;
      q.out_pool = pool;
      CK(svf::launch_query_keys(q.queries, j.stride, q.qids, j.dim, ntop, j.seed, qkey, st));
      q.qkey = qkey;
      CK(svf::launch_search(q, j.prec, st));
      CK(svf::launch_topup_merge(a, pool, j.Lins, (int)first, ntop, st));
    }
    svf::PruneArgs pa{};
    pa.cand = cand;
    pa.cstride = cap;
    pa.cap = cap;
    pa.graph = j.graph;
    pa.fwd = nullptr;
    pa.n_old = (int32_t)j.n_slots;
    pa.R = R;
    pa.out_ids = rows + first * R;
    pa.out_d = rows_d + first * R;
    pa.nlists = count;
    pa.skip = mcount;                        // -1: pruned by the long-list kernels
    CK(svf::launch_prune_lists(pa, st));
  }
  CK(hipStreamSynchronize(st));
  *n_aff_out = n_aff;
  return SVF_OK;
}

// Write n rows computed by a repair pass into the live graph.
int commit_repaired(svf_index* ix, const int32_t* list, int n, const int32_t* rows,
                    const float* rows_d, hipStream_t st) {
  if (n <= 0) return SVF_OK;
  if (int32_t* e = kept_indegree(ix))
    CK(svf::launch_indegree_rows_delta(ix->graph, list, n, rows, ix->R, e, st));
  CK(svf::launch_commit_rows(list, n, rows, rows_d, ix->R, ix->graph, ix->edge_d, st));
  ++ix->graph_epoch;
  return row_scales_rows(ix, list, 0, n, st);
}

// Repair (consolidate = 0) or consolidation (1) of the live graph.
int repair(svf_index* ix, int consolidate) {
  hipStream_t st = ix->stream;
  if (consolidate) ++ix->st.consolidations;
  CK(hipEventRecord(ix->ev0, st));
  int32_t n_aff = 0;
  int rc = repair_compute(repair_job(ix), consolidate, ix->rs, st, &n_aff);
  if (rc) return rc;
  ix->st.last_repaired = n_aff;
  if (n_aff == 0) {
    ix->st.del_repair_ms = 0;
    return SVF_OK;
  }
  if ((rc = commit_repaired(ix, ix->rs.list.as<int32_t>(), n_aff, ix->rs.rows.as<int32_t>(),
                            ix->rs.rows_d.as<float>(), st)))
    return rc;
  CK(hipEventRecord(ix->ev1, st));
  CK(hipStreamSynchronize(st));
  ix->st.del_repair_ms = elapsed(ix->ev0, ix->ev1);
  return SVF_OK;
}

// ---- consolidation in the background (Sec. 5.3) ------------------------------
// bg_begin copies the live rows, edge distances and alive bits and starts a
// host thread that runs the consolidation on that snapshot on its own
// stream.  Meanwhile the live graph keeps changing; every insertion batch
// appends its forward rows to a log.  bg_merge waits for the thread, writes
// the consolidated rows into the live graph, then re-prunes each rewritten
// row with the edges that insertions since the snapshot gave it (the log's
// pairs whose target is a rewritten row), as a reverse-edge pass reading
// the rows as they stand after the first step.  Rows of vertices inserted
// since the snapshot, and rows the consolidation did not rewrite, keep their
// live state.
void bg_join(svf_index* ix) {
  if (ix->bg.th.joinable()) ix->bg.th.join();
}

int bg_begin(svf_index* ix) {
  svf::BgConsolidation& B = ix->bg;
  hipStream_t st = ix->stream;
  if (!B.st) CK(hipStreamCreateWithFlags(&B.st, hipStreamNonBlocking));
  const int64_t n = ix->n_slots, R = ix->R, words = (n + 31) / 32;
  int32_t* g;
  float* e;
  uint32_t* al;
  int rc;
  if ((rc = scratch(B.graph, std::max<int64_t>(n * R, 1), &g)) ||
      (rc = scratch(B.edge_d, std::max<int64_t>(n * R, 1), &e)) ||
      (rc = scratch(B.alive, std::max<int64_t>(words, 1), &al)))
    return rc;
  CK(hipMemcpyAsync(g, ix->graph, n * R * 4, hipMemcpyDeviceToDevice, st));
  CK(hipMemcpyAsync(e, ix->edge_d, n * R * 4, hipMemcpyDeviceToDevice, st));
  CK(hipMemcpyAsync(al, ix->alive, words * 4, hipMemcpyDeviceToDevice, st));
  CK(hipStreamSynchronize(st));
  RepairJob j = repair_job(ix);
  j.graph = g;
  j.edge_d = e;
  j.alive = al;
  j.proto.graph = g;
  j.proto.alive = al;
  j.proto.nscale = nullptr;                 // the live rows' scales, not the snapshot's
  B.n0 = n;
  B.log_n = 0;
  B.n_aff = 0;
  B.rc = 0;
  B.err.clear();
  B.done = false;
  B.active = true;
  const int dev = ix->device;
  B.th = std::thread([&B, j, dev]() {
    int32_t na = 0;
    int rc2 = hipSetDevice(dev) == hipSuccess ? repair_compute(j, 1, B.rs, B.st, &na) : SVF_E_DEVICE;
    B.n_aff = na;
    B.rc = rc2;
    if (rc2) B.err = g_err;
    B.done = true;
  });
  return SVF_OK;
}

// Append the forward rows of an insertion batch (ids B.n0 + B.log_n on) to the log.
int bg_log(svf_index* ix, const int32_t* fwd, const float* fwd_d, int64_t b, hipStream_t st) {
  svf::BgConsolidation& B = ix->bg;
  const int64_t R = ix->R;
  if (B.log_n + b > B.log_cap) {
    const int64_t cap = std::max<int64_t>(B.log_n + b, 2 * B.log_cap);
    svf::DevBuf ni, nd;
    CK(ni.ensure(cap * R * 4));
    CK(nd.ensure(cap * R * 4));
    if (B.log_n) {
      CK(hipMemcpyAsync(ni.p, B.log_ids.p, B.log_n * R * 4, hipMemcpyDeviceToDevice, st));
      CK(hipMemcpyAsync(nd.p, B.log_d.p, B.log_n * R * 4, hipMemcpyDeviceToDevice, st));
      CK(hipStreamSynchronize(st));
    }
    std::swap(B.log_ids.p, ni.p);
    std::swap(B.log_ids.bytes, ni.bytes);
    std::swap(B.log_d.p, nd.p);
    std::swap(B.log_d.bytes, nd.bytes);
    B.log_cap = cap;
  }
  CK(hipMemcpyAsync(B.log_ids.as<int32_t>() + B.log_n * R, fwd, b * R * 4, hipMemcpyDeviceToDevice, st));
  CK(hipMemcpyAsync(B.log_d.as<float>() + B.log_n * R, fwd_d, b * R * 4, hipMemcpyDeviceToDevice, st));
  B.log_n += b;
  return SVF_OK;
}

int bg_merge(svf_index* ix) {
  svf::BgConsolidation& B = ix->bg;
  if (!B.active) return SVF_OK;
  bg_join(ix);
  B.active = false;
  if (B.rc) {
    B.log_n = 0;
    return fail(B.rc, "background consolidation: " + B.err);
  }
  hipStream_t st = ix->stream;
  const int R = ix->R;
  const int32_t n_aff = B.n_aff;
  ix->st.last_repaired = n_aff;
  ++ix->st.consolidations;
  int rc;
  if (n_aff > 0) {
    const int32_t* list = B.rs.list.as<int32_t>();
    if ((rc = commit_repaired(ix, list, n_aff, B.rs.rows.as<int32_t>(), B.rs.rows_d.as<float>(), st)))
      return rc;
  }
  if (n_aff > 0 && B.log_n > 0) {
    const int64_t words = (ix->n_slots + 31) / 32;
    uint32_t* mask;
    int32_t* cnt;
    if ((rc = scratch_grow(B.mask, words, &mask)) || (rc = scratch_grow(ix->s_misc[2], 8, &cnt))) return rc;
    CK(svf::launch_fill_u32(mask, words, 0u, st));
    CK(svf::launch_mark_list(B.rs.list.as<int32_t>(), n_aff, mask, st));
    svf::ReverseArgs ra{};
    ra.fwd_ids = B.log_ids.as<int32_t>();
    ra.fwd_d = B.log_d.as<float>();
    ra.b = (int)B.log_n;
    ra.R = R;
    ra.n0 = (int32_t)B.n0;
    ra.rows_below = (int32_t)ix->n_slots;
    ra.tmask = mask;
    ra.tcount = tcount(ix);
    ra.tidx = tidx(ix);
    ra.graph = ix->graph;
    ra.edge_d = ix->edge_d;
    ra.alive = ix->alive;
    ra.cap = prune_cap(ix);
    const int64_t npairs = B.log_n * R;
    if ((rc = scratch(ix->s_misc[3], npairs, &ra.tlist))) return rc;
    ra.n_targets = cnt;
    CK(svf::launch_fill_u32(cnt, 1, 0u, st));
    CK(svf::launch_reverse_count(ra, st));
    int32_t n_targets = 0;
    CK(hipMemcpyAsync(&n_targets, cnt, 4, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    const size_t nt = (size_t)n_targets;
    if ((rc = scratch_grow(ix->s_misc[4], nt + 1, &ra.off)) ||
        (rc = scratch_grow(ix->s_misc[5], nt + 2 + nt / 1024 + 2, &ra.cursor)) ||
        (rc = scratch(ix->s_misc[6], npairs, &ra.inc)) ||
        (rc = scratch_grow(ix->s_misc[7], nt * R, &ra.trow)) ||
        (rc = scratch_grow(ix->s_misc[8], nt * R, &ra.trow_d)))
      return rc;
    CK(svf::launch_reverse_scan_scatter(ra, n_targets, st));
    if ((rc = reverse_prune_all(ix, ra, n_targets, st))) return rc;
    if (int32_t* e = kept_indegree(ix))
      CK(svf::launch_indegree_rows_delta(ix->graph, ra.tlist, n_targets, ra.trow, R, e, st));
    svf::ReverseArgs only_targets = ra;
    only_targets.b = 0;                       // the logged rows are live already
    CK(svf::launch_commit_batch(only_targets, n_targets, ix->graph, ix->edge_d, ix->alive, st));
    ++ix->graph_epoch;
    if ((rc = row_scales_rows(ix, ra.tlist, 0, n_targets, st))) return rc;
  }
  CK(hipStreamSynchronize(st));
  B.log_n = 0;
  return SVF_OK;
}

int search_impl(svf_index* ix, const float* d_q, int64_t nq, int k, int beam, int32_t* d_ids,
                float* d_d, int32_t* d_nd, int32_t* d_ne, hipStream_t st, uint64_t* ws_qkey) {
  if (nq == 0) return SVF_OK;
  uint64_t* qkey = ws_qkey;
  unsigned long long* tot = nullptr;   // batch totals are kept only with the index's own buffers
  int rc;
  if (!ws_qkey && ((rc = scratch(ix->s_qkey, nq, &qkey)) || (rc = scratch(ix->s_tot, 3, &tot))))
    return rc;
  if (ix->n_slots == 0) {
    // nothing indexed: every result is padding
    CK(svf::launch_fill_u32(d_ids, nq * k, 0xffffffffu, st));
    CK(svf::launch_fill_u32(d_d, nq * k, 0x7f800000u, st));
    if (d_nd) CK(svf::launch_fill_u32(d_nd, nq, 0u, st));
    if (d_ne) CK(svf::launch_fill_u32(d_ne, nq, 0u, st));
    return SVF_OK;
  }
  svf::SearchArgs a = base_args(ix);
  set_beam(a, ix, beam);
  a.k = k;
  a.queries = d_q;
  a.qstride = ix->dim;
  a.nq = (int)nq;
  // the totals start at zero before any kernel of this batch counts into them
  // (the gating below counts its fallbacks)
  if (tot) CK(svf::launch_fill_u32(tot, 6, 0u, st));
  if (ix->opt.use_model && ix->model) {
    if (ws_qkey) return fail(SVF_E_INVAL, "the learned form needs the index's own workspace");
    float* z;
    int32_t *qe, *qm;
    if ((rc = scratch(ix->s_z, (size_t)nq * (ix->model_nc + 1), &z)) ||
        (rc = scratch(ix->s_qentry, nq, &qe)) || (rc = scratch(ix->s_qmax, nq, &qm)))
      return rc;
    CK(ix->model->forward(d_q, nq, z, st));
    CK(svf::launch_model_decide(z, nq, ix->model_nc, (float)ix->opt.model_conf,
                                (float)ix->opt.model_stop_scale, ix->opt.model_min_iters, qe, qm,
                                tot + 2, st));
    a.entry_lists = ix->entry_lists.as<int32_t>();
    a.entry_cap = ix->entry_cap;
    a.q_entry = qe;
    a.q_max_iters = qm;
  }
  a.out_ids = d_ids;
  a.out_d = d_d;
  a.n_dist = d_nd;
  a.n_exp = d_ne;
  a.totals = tot;
  if (ix->tier.on) {
    if (ws_qkey) return fail(SVF_E_INVAL, "the tiered store needs the index's own workspace");
    svf::TierState& T = ix->tier;
    unsigned long long* cnt;
    if ((rc = scratch(T.trace, (size_t)nq * T.trace_cap, &a.trace)) ||
        (rc = scratch(T.trace_n, nq, &a.trace_n)) || (rc = scratch(T.counts, 2, &cnt)))
      return rc;
    a.trace_cap = T.trace_cap;
    a.tier_counts = cnt;
    CK(svf::launch_fill_u32(cnt, 4, 0u, st));
  }
  CK(svf::launch_query_keys(d_q, ix->dim, nullptr, ix->dim, a.nq, ix->opt.seed, qkey, st));
  a.qkey = qkey;
  CK(hipEventRecord(ix->ev0, st));
  // Alg. 1's X_CPU: with cache_cpu_miss the misses of an FP32 traversal of
  // the tiered store are computed on the host cores (random entry points,
  // one parent per iteration; other forms read misses over the host link)
  if (ix->tier.on && ix->opt.cache_cpu_miss && ix->veclp_prec == 0 && !a.q_entry && a.width == 1) {
    if ((rc = co_search(ix, a, d_q, nq, st))) return rc;
  } else {
    CK(svf::launch_search(a, ix->veclp_prec, st));
  }
  CK(hipEventRecord(ix->ev1, st));
  ix->st.last_queries = nq;
  return SVF_OK;
}

// Insert n device-resident vectors.  Into an empty index this is the build
// rule: a seed of min(n, 4R) vectors, then batches of
// min(insert_batch_max, ceil(n_alive / 8)); otherwise batches of
// insert_batch_max.
int insert_stream(svf_index* ix, const float* d, int64_t n, int32_t* d_out_ids, int32_t* h_out_ids) {
  int64_t done = 0;
  const bool grow = ix->n_slots == 0;
  int rc = reserve(ix, ix->n_slots + n);
  if (rc) return rc;
  if (grow && n > 0) {
    const int64_t s0 = std::min<int64_t>(n, 4 * ix->R);
    rc = insert_batch(ix, d, s0, d_out_ids, h_out_ids);
    if (rc) return rc;
    done = s0;
  }
  while (done < n) {
    int64_t b = std::min<int64_t>(ix->opt.insert_batch_max, n - done);
    if (grow) b = std::min<int64_t>(b, (ix->n_alive + 7) / 8);
    rc = insert_batch(ix, d + done * ix->dim, b, d_out_ids ? d_out_ids + done : nullptr,
                      h_out_ids ? h_out_ids + done : nullptr);
    if (rc) return rc;
    done += b;
  }
  return SVF_OK;
}

int check_search_args(const svf_index* ix, int64_t nq, int k, int beam) {
  if (!ix) return fail(SVF_E_INVAL, "null index");
  if (nq < 0 || nq > (1 << 25)) return fail(SVF_E_INVAL, "nq must be in [0, 2^25]");
  if (k < 1) return fail(SVF_E_INVAL, "k must be >= 1");
  if (beam < k) return fail(SVF_E_INVAL, "beam must be >= k");
  if (beam > kMaxSearchBeam) return fail(SVF_E_INVAL, "beam must be <= 1024");
  return SVF_OK;
}

// A float is finite unless its exponent bits are all ones (inf or NaN).  The
// test runs over blocks of 4096 values with a branch-free OR of the exponent
// tests, which the compiler vectorizes, and stops at the first bad block.
bool all_finite(const float* p, int64_t n) {
  constexpr int64_t kBlock = 4096;
  for (int64_t i0 = 0; i0 < n; i0 += kBlock) {
    const int64_t i1 = i0 + kBlock < n ? i0 + kBlock : n;
    uint32_t bad = 0;
    for (int64_t i = i0; i < i1; ++i) {
      uint32_t u;
      std::memcpy(&u, p + i, 4);
      bad |= (uint32_t)((u & 0x7f800000u) == 0x7f800000u);
    }
    if (bad) return false;
  }
  return true;
}

void finish_search_stats(svf_index* ix) {
  unsigned long long tot[3] = {0, 0, 0};
  if (ix->s_tot.p && hipMemcpy(tot, ix->s_tot.p, sizeof tot, hipMemcpyDeviceToHost) == hipSuccess) {
    ix->st.last_n_dist = (int64_t)tot[0];
    ix->st.last_n_exp = (int64_t)tot[1];
    ix->st.last_model_fallback = (ix->opt.use_model && ix->model) ? (int64_t)tot[2] : 0;
  }
  ix->st.last_search_ms = elapsed(ix->ev0, ix->ev1);
}

// Mark ids deleted (host ids, validated against n_slots first), then repair
// or consolidate.  The caller holds the index.
int delete_ids(svf_index* ix, const int32_t* ids, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (ids[i] < 0 || ids[i] >= ix->n_slots) return fail(SVF_E_NOTFOUND, "id out of range");
  if (n == 0) return SVF_OK;
  hipStream_t st = ix->stream;
  int32_t *d, *cnt;
  int rc;
  if ((rc = scratch_grow(ix->s_misc[9], n, &d)) || (rc = scratch_grow(ix->s_tot, 2, &cnt))) return rc;
  CK(hipEventRecord(ix->ev0, st));
  CK(hipMemcpyAsync(d, ids, n * 4, hipMemcpyHostToDevice, st));
  CK(svf::launch_fill_u32(cnt, 1, 0u, st));
  CK(svf::launch_mark_deleted(d, n, ix->alive, cnt, ix->graph, ix->R, kept_indegree(ix), st));
  int32_t newly = 0;
  CK(hipMemcpyAsync(&newly, cnt, 4, hipMemcpyDeviceToHost, st));
  CK(hipEventRecord(ix->ev1, st));
  CK(hipStreamSynchronize(st));
  ix->st.del_mark_ms = elapsed(ix->ev0, ix->ev1);
  ++ix->graph_epoch;
  if ((rc = tier_release(ix, ids, n))) return rc;
  if (ix->alive_at_consolidate == 0) ix->alive_at_consolidate = ix->n_alive;
  ix->n_alive -= newly;
  ix->deleted_since += newly;
  if (newly == 0) return SVF_OK;
  const bool due = ix->opt.consolidate_frac > 0 &&
                   (double)ix->deleted_since >= ix->opt.consolidate_frac * (double)ix->alive_at_consolidate;
  const bool async = ix->opt.consolidate_async && !ix->tier.on;
  if (due && async && !ix->bg.active) {
    rc = bg_begin(ix);                     // the consolidation runs on a snapshot
    ix->deleted_since = 0;
    ix->alive_at_consolidate = ix->n_alive;
  } else if (due && !async) {
    if ((rc = bg_merge(ix))) return rc;
    rc = repair(ix, 1);
    ix->deleted_since = 0;
    ix->alive_at_consolidate = ix->n_alive;
  } else if (ix->opt.localized_repair) {
    rc = repair(ix, 0);                    // (a due consolidation waits for the pending one)
  }
  return rc;
}

// ---- tiered store: slots follow deletions and insertions ---------------------
// A deleted vector leaves the cache at once and its slot becomes free; new
// vectors take free slots in id order (write-allocate), so a cache that
// holds every live vector keeps doing so under updates.  While the serving
// loop runs the cache does not change (searches of other streams may be
// reading it).
int tier_release(svf_index* ix, const int32_t* ids, int64_t n) {
  svf::TierState& T = ix->tier;
  if (T.on && ix->server && n > 0) T.dead_residents = true;   // kept until evicted
  if (!T.on || ix->server || n == 0) return SVF_OK;
  std::vector<int32_t> place;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t x = ids[i];
    const int32_t s_ = T.where[x];
    if (s_ < 0) continue;
    T.where[x] = -1;
    T.slot_id[s_] = -1;
    T.ref[s_] = 0;
    T.free_slots.push_back(s_);
    place.insert(place.end(), {s_, -1, x});
  }
  const int64_t placed = T.last_placed;
  const int rc = tier_apply(ix, place, ix->stream);
  T.last_placed = placed;
  return rc;
}

int tier_admit(svf_index* ix, int64_t id0, int64_t n) {
  svf::TierState& T = ix->tier;
  if (!T.on || ix->server || T.building || n == 0) return SVF_OK;
  std::vector<int32_t> place;
  for (int64_t x = id0; x < id0 + n; ++x) {
    const int64_t slot = T.take_slot();
    if (slot < 0) break;
    T.occupy(slot, (int32_t)x);
    place.insert(place.end(), {(int32_t)slot, (int32_t)x, -1});
  }
  T.promotions += place.size() / 3;
  const int64_t placed = T.last_placed;
  const int rc = tier_apply(ix, place, ix->stream);
  T.last_placed = placed;
  return rc;
}

// ---- tiered store: placement after each query batch ------------------------
// The batched form of workload-aware placement (Sec. 4.3, Alg. 2, Eq. 2): per
// batch F_recent halves and counts the batch's expansion trace (queries in
// order, each query's expanded vertices in order); accesses to cached vectors
// are hits and set their slot's reference bit; the distinct missed vectors
// with F_lambda = alpha F_recent + beta log(1 + E_in) above theta, by
// (F_lambda desc, id asc), at most promote_max of them, are placed one after
// another: into a free slot, else over Alg. 2's clock (WavpSweep): F_min over
// the residents with a clear reference bit, the hand clearing set bits up to
// the first clear slot holding F_min, which is replaced, the hand staying on
// it.  With cache_theta_adapt > 1, theta follows the batch's miss rate and
// the mean F_lambda of its missed vectors (Sec. 4.4) before the placements.
int tier_refresh_indegree(svf_index* ix, hipStream_t st) {
  svf::TierState& T = ix->tier;
  const bool recount = !T.e_in_valid;
  if (!recount && !T.verify_indegree && T.e_in_epoch == ix->graph_epoch && T.e_in_n >= ix->n_slots)
    return SVF_OK;
  const int64_t cap = std::max<int64_t>(ix->cap, 1);
  int32_t* d;
  int rc = scratch(T.e_in_d, cap, &d);
  if (rc) return rc;
  CK(T.e_in.ensure(cap * 4));
  if (recount) {
    CK(svf::launch_fill_u32(d, cap, 0u, st));
    CK(svf::launch_indegree(ix->graph, ix->alive, ix->n_slots, ix->R, d, st));
    T.e_in_valid = true;
  }
  CK(hipMemcpyAsync(T.e_in.p, d, ix->n_slots * 4, hipMemcpyDeviceToHost, st));
  if (T.C > 0 && T.sdeg) {                  // the slots' in-degrees, in slot order
    int32_t* sd;
    if ((rc = scratch(T.sdeg_d, (size_t)T.C, &sd))) return rc;
    CK(svf::launch_fill_u32(reinterpret_cast<uint32_t*>(sd), T.C, 0u, st));
    CK(svf::launch_slot_indegree(T.map, d, ix->n_slots, sd, st));
    CK(hipMemcpyAsync(T.sdeg, sd, T.C * 4, hipMemcpyDeviceToHost, st));
  }
  if (!recount && T.verify_indegree) {
    int32_t* chk;
    if ((rc = scratch(T.e_in_chk, cap, &chk))) return rc;
    CK(svf::launch_indegree(ix->graph, ix->alive, ix->n_slots, ix->R, chk, st));
    std::vector<int32_t> want(ix->n_slots);
    CK(hipMemcpyAsync(want.data(), chk, ix->n_slots * 4, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    for (int64_t i = 0; i < ix->n_slots; ++i)
      if (want[i] != T.in_degree((int32_t)i)) return fail(SVF_E_INTERNAL, "kept in-degree differs from a recount");
  }
  CK(hipStreamSynchronize(st));
  T.e_in_n = ix->n_slots;
  T.e_in_epoch = ix->graph_epoch;
  return SVF_OK;
}

// Move a batch's placements (slot, new id, evicted id or -1, in decision
// order) to the device.  A slot can change hands more than once in a batch
// (a vector placed early in the batch evicted by a later one), and the
// placement kernel runs all entries at once, so the list is first reduced to
// one entry per slot: the occupant at the start of the batch leaves, the
// last one placed arrives; vectors placed and evicted within the batch never
// reach the device map.
int tier_apply(svf_index* ix, const std::vector<int32_t>& place, hipStream_t st) {
  svf::TierState& T = ix->tier;
  const int np = (int)(place.size() / 3);
  T.last_placed = np;
  if (np == 0) return SVF_OK;
  std::vector<int32_t> net;
  net.reserve(place.size());
  std::vector<std::pair<int32_t, int32_t>> idx;   // (slot, position in net)
  idx.reserve(np);
  for (int p = 0; p < np; ++p) idx.emplace_back(place[3 * p], p);
  std::stable_sort(idx.begin(), idx.end(),
                   [](const std::pair<int32_t, int32_t>& a, const std::pair<int32_t, int32_t>& b) {
                     return a.first < b.first;
                   });
  for (size_t i = 0; i < idx.size();) {
    size_t j = i;
    while (j + 1 < idx.size() && idx[j + 1].first == idx[i].first) ++j;
    const int first = idx[i].second, lastp = idx[j].second;
    net.insert(net.end(), {place[3 * first], place[3 * lastp + 1], place[3 * first + 2]});
    i = j + 1;
  }
  const int nn = (int)(net.size() / 3);
  int32_t* d;
  int rc = scratch(T.place, net.size(), &d);
  if (rc) return rc;
  CK(hipMemcpyAsync(d, net.data(), net.size() * 4, hipMemcpyHostToDevice, st));
  CK(svf::launch_place(d, nn, T.segs(), T.cache, ix->stride, T.map, st));
  CK(hipStreamSynchronize(st));
  return SVF_OK;
}

// F_recent halves once per placement batch; a vertex's value is brought up
// to date only when it is used.  Repeated halving is an exact power-of-two
// scaling while the result stays a normal double, so whole runs of halvings
// are one ldexp; below the normal range they are applied one by one, with
// the rounding each single halving has.
double halve_times(double v, int64_t k) {
  if (k <= 0) return v;
  uint64_t u;
  std::memcpy(&u, &v, 8);
  const int64_t eb = (int64_t)((u >> 52) & 0x7ff);
  if (eb != 0x7ff && eb > k) {               // normal in and out: lower the exponent field
    u -= (uint64_t)k << 52;
    std::memcpy(&v, &u, 8);
    return v;
  }
  while (k > 0 && v != 0.0) {
    int e;
    (void)std::frexp(v, &e);                 // |v| = m 2^e, m in [0.5, 1)
    const int64_t room = (int64_t)e + 1021;  // halvings that keep |v| >= 2^-1022
    if (room > 0) {
      const int64_t j = std::min(k, room);
      v = std::ldexp(v, -(int)j);
      k -= j;
    } else {
      v *= 0.5;
      --k;
    }
  }
  return v;
}
double fr_now(const svf::TierState& T, int32_t x) {
  return halve_times(T.fr[x].v, T.batch - T.fr[x].stamp);
}

// The classic replacement policies (LRU, LFU, LRFU) in the batched form: the
// batch's missed vertices, most important first (ties by id), at most
// promote_max, each take a free slot or the slot of the least important
// resident vertex, which is always evicted.  Importance: last access (LRU),
// accesses so far (LFU), F_recent (LRFU), ties by id (the larger id is the
// less important); scores do not change while a batch is placed.  With m
// candidates at most m residents leave, and each one is the least important
// of those left, so a heap over the m least important residents plus the
// vertices placed in this batch yields the same evictions as one over all.
template <class Key>
int place_classic(svf_index* ix, std::vector<int32_t>& order, Key key, hipStream_t st) {
  svf::TierState& T = ix->tier;
  using E = std::pair<decltype(key(0)), int32_t>;
  auto more = [](const E& a, const E& b) {            // a more important than b
    return a.first > b.first || (a.first == b.first && a.second < b.second);
  };
  std::vector<E> cand;
  cand.reserve(order.size());
  for (const int32_t x : order) cand.emplace_back(key(x), x);
  if ((int64_t)cand.size() > T.promote_max) {
    std::nth_element(cand.begin(), cand.begin() + T.promote_max, cand.end(), more);
    cand.resize(T.promote_max);
  }
  std::sort(cand.begin(), cand.end(), more);
  const int64_t m = (int64_t)cand.size();
  std::vector<E> heap;                                // least important on top
  const bool evicting = m > T.free_count();
  if (evicting) {
    heap.reserve(T.used + m);
    for (int64_t s_ = 0; s_ < T.used; ++s_)
      if (T.slot_id[s_] >= 0) heap.emplace_back(key(T.slot_id[s_]), T.slot_id[s_]);
    if ((int64_t)heap.size() > m) {
      std::nth_element(heap.begin(), heap.end() - m, heap.end(), more);
      heap.erase(heap.begin(), heap.end() - m);
    }
    std::make_heap(heap.begin(), heap.end(), more);
  }
  std::vector<int32_t> place;
  for (const E& c : cand) {
    const int32_t x = c.second;
    const int64_t slot = T.take_slot();
    if (slot >= 0) {
      T.occupy(slot, x);
      place.insert(place.end(), {(int32_t)slot, x, -1});
      if (evicting) {
        heap.push_back(c);
        std::push_heap(heap.begin(), heap.end(), more);
      }
      continue;
    }
    if (T.C == 0) break;
    std::pop_heap(heap.begin(), heap.end(), more);
    const int32_t y = heap.back().second;
    heap.pop_back();
    const int32_t s_ = T.where[y];
    T.where[y] = -1;
    T.occupy(s_, x);
    place.insert(place.end(), {s_, x, y});
    ++T.evictions;
    heap.push_back(c);
    std::push_heap(heap.begin(), heap.end(), more);
  }
  T.promotions += place.size() / 3;
  return tier_apply(ix, place, st);
}

int tier_place_classic(svf_index* ix, std::vector<int32_t>& order, hipStream_t st) {
  svf::TierState& T = ix->tier;
  if (T.policy == 1) return place_classic(ix, order, [&](int32_t x) { return T.last[x]; }, st);
  if (T.policy == 2) return place_classic(ix, order, [&](int32_t x) { return T.freq[x]; }, st);
  return place_classic(ix, order, [&](int32_t x) { return fr_now(T, x); }, st);
}

int tier_after_batch(svf_index* ix, int64_t nq, hipStream_t st) {
  svf::TierState& T = ix->tier;
  using clk = std::chrono::steady_clock;
  auto ms_since = [](clk::time_point t0) {
    return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  };
  auto tp = clk::now();
  ix->st.place_indeg_ms = ix->st.place_walk_ms = ix->st.place_evict_ms = ix->st.place_apply_ms = 0;
  const int cap = T.trace_cap;
  const int64_t n = ix->n_slots;
  const int64_t words = (n + 31) / 32;
  // On the GPU: per-vertex access counts, the touched bitmap (and for LRU the
  // last positions), then the list of touched vertices in id order; only that
  // list comes back to the host.
  const bool lru = T.policy == 1;
  int32_t *cnt_d, *lastpos_d = nullptr, *blk_d;
  uint32_t* touched_d;
  const int64_t nb = svf::touched_blocks(words);
  int rc;
  if ((rc = scratch_grow(T.acc_cnt, n, &cnt_d)) || (rc = scratch_grow(T.touched, words, &touched_d)) ||
      (lru && (rc = scratch_grow(T.lastpos, n, &lastpos_d))) || (rc = scratch_grow(T.blk, 2 * nb + 2, &blk_d)))
    return rc;
  CK(T.blk_h.ensure((nb + 1) * 8));
  CK(T.alive_h.ensure((words + 1) * 4));
  CK(svf::launch_fill_u32(cnt_d, n, 0u, st));
  CK(svf::launch_fill_u32(touched_d, words, 0u, st));
  if (lru) CK(svf::launch_fill_u32(lastpos_d, n, 0xffffffffu, st));
  CK(svf::launch_trace_count(T.trace.as<int32_t>(), T.trace_n.as<int32_t>(), (int)nq, cap, cnt_d,
                             touched_d, lastpos_d, st));
  CK(svf::launch_touched_count(touched_d, words, blk_d, st));
  unsigned long long gcnt[2] = {0, 0};
  int32_t* btot = T.blk_h.as<int32_t>();
  uint32_t* bits = T.alive_h.as<uint32_t>();
  CK(hipMemcpyAsync(btot, blk_d, nb * 4, hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(gcnt, T.counts.p, sizeof gcnt, hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(bits, ix->alive, words * 4, hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  bits[words] = 0u;
  int32_t* boff = btot + nb;                    // exclusive offsets, then the total
  int64_t total = 0;
  for (int64_t b = 0; b < nb; ++b) {
    boff[b] = (int32_t)total;
    total += btot[b];
  }
  int32_t *lid, *lcnt, *llast = nullptr;
  if ((rc = scratch_grow(T.lst_id, total + 1, &lid)) || (rc = scratch_grow(T.lst_cnt, total + 1, &lcnt)) ||
      (lru && (rc = scratch_grow(T.lst_last, total + 1, &llast))))
    return rc;
  CK(T.lst_id_h.ensure((total + 1) * 4));
  CK(T.lst_cnt_h.ensure((total + 1) * 4));
  if (lru) CK(T.lst_last_h.ensure((total + 1) * 4));
  CK(hipMemcpyAsync(blk_d + nb, boff, nb * 4, hipMemcpyHostToDevice, st));
  CK(svf::launch_touched_list(touched_d, words, blk_d + nb, cnt_d, lastpos_d, lid, lcnt, llast, st));
  const int32_t* tid = T.lst_id_h.as<int32_t>();
  const int32_t* tcnt = T.lst_cnt_h.as<int32_t>();
  const int32_t* tlast = lru ? T.lst_last_h.as<int32_t>() : nullptr;
  CK(hipMemcpyAsync(T.lst_id_h.p, lid, total * 4, hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(T.lst_cnt_h.p, lcnt, total * 4, hipMemcpyDeviceToHost, st));
  if (lru) CK(hipMemcpyAsync(T.lst_last_h.p, llast, total * 4, hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  ix->st.place_count_ms = ms_since(tp);
  tp = clk::now();
  rc = tier_refresh_indegree(ix, st);
  if (rc) return rc;
  ix->st.place_indeg_ms = ms_since(tp);
  tp = clk::now();
  T.gather_hits += gcnt[0];
  T.gather_misses += gcnt[1];
  auto alive = [&](int32_t x) { return ((bits[x >> 5] >> (x & 31)) & 1u) != 0; };
  (void)T.log1p_deg(0);                     // the table is filled before the threads read it
  auto lg = [&](int32_t x) { return T.beta * T.log1p_deg(T.in_degree(x)); };
  ++T.batch;
  // every touched vertex in id order: F_recent halves, then gains one per
  // access; accesses of cached vertices are hits and set their slot's
  // reference bit; uncached vertices above theta become candidates.  The
  // vertices are independent, so contiguous ranges of the list run on
  // separate threads and their candidates are joined in order.
  const int nthr = (int)std::max<int64_t>(1, std::min<int64_t>({16, (total + 16383) / 16384,
                                                                 (int64_t)std::thread::hardware_concurrency()}));
  // Candidates are taken against theta after the adaptation, which needs the
  // whole batch: each thread keeps the prediction of every missed alive
  // vertex of its range, in id order.
  std::vector<std::vector<std::pair<double, int32_t>>> tcand(nthr);
  std::vector<std::vector<int32_t>> tmissed(nthr);
  std::vector<int64_t> thits(nthr, 0), tacc(nthr, 0);
  const int32_t* indeg_h = T.e_in.as<int32_t>();
  auto work = [&](int t) {
    const int64_t lo = total * t / nthr, hi = total * (t + 1) / nthr;
    int64_t h = 0, a = 0;
    for (int64_t i = lo; i < hi; ++i) {
      if (i + 32 < hi) {               // the touched ids are sparse: request ahead
        const int32_t xa = tid[i + 32];
        __builtin_prefetch(&T.fr[xa]);
        __builtin_prefetch(&T.freq[xa]);
        __builtin_prefetch(&T.where[xa]);
        __builtin_prefetch(&bits[xa >> 5]);
        __builtin_prefetch(&indeg_h[xa]);
      }
      const int32_t x = tid[i];
      double v = fr_now(T, x);
      const int32_t c = tcnt[i];
      for (int32_t k = 0; k < c; ++k) v += 1.0;
      a += c;
      T.fr[x].v = v;
      T.fr[x].stamp = T.batch;
      T.freq[x] += c;
      if (lru) T.last[x] = ((T.batch - 1) << 40) + tlast[i];
      if (T.where[x] >= 0) {
        h += c;
        T.ref[T.where[x]] = 1;
        T.sfr[T.where[x]] = T.fr[x];
      } else if (alive(x)) {
        if (T.policy == 0) tcand[t].emplace_back(T.alpha * v + lg(x), x);
        else tmissed[t].push_back(x);
      }
    }
    thits[t] = h;
    tacc[t] = a;
  };
  if (nthr == 1) {
    work(0);
  } else {
    std::vector<std::thread> pool;
    for (int t = 1; t < nthr; ++t) pool.emplace_back(work, t);
    work(0);
    for (auto& th : pool) th.join();
  }
  int64_t hits = 0, acc = 0;
  std::vector<std::pair<double, int32_t>> cand;
  std::vector<int32_t> missed;
  for (int t = 0; t < nthr; ++t) {
    hits += thits[t];
    acc += tacc[t];
    missed.insert(missed.end(), tmissed[t].begin(), tmissed[t].end());
  }
  T.last_trace_hits = hits;
  if (T.policy != 0) {
    ix->st.place_walk_ms = ms_since(tp);
    return tier_place_classic(ix, missed, st);
  }
  if (T.adapt > 1.0 && acc > 0) {
    // Sec. 4.4: theta rises when the miss rate and the mean prediction of the
    // missed vectors both rise, and falls back (not below where it started)
    // when both fall.  The mean is summed in id order.
    double sum = 0.0;
    int64_t cnt = 0;
    for (int t = 0; t < nthr; ++t)
      for (const auto& c : tcand[t]) { sum += c.first; ++cnt; }
    const double mean = cnt ? sum / (double)cnt : 0.0;
    const int64_t miss = acc - hits;
    if (T.have_prev) {
      const bool rose = (__int128)miss * T.prev_acc > (__int128)T.prev_miss * acc;
      const bool fell = (__int128)miss * T.prev_acc < (__int128)T.prev_miss * acc;
      if (rose && mean > T.prev_mean) T.theta *= T.adapt;
      else if (fell && mean < T.prev_mean) T.theta = std::max(T.theta0, T.theta / T.adapt);
    }
    T.have_prev = true;
    T.prev_miss = miss;
    T.prev_acc = acc;
    T.prev_mean = mean;
  }
  auto better = [](const std::pair<double, int32_t>& a, const std::pair<double, int32_t>& b) {
    return a.first > b.first || (a.first == b.first && a.second < b.second);
  };
  // The placements are the promote_max best candidates above theta in the
  // (F_lambda desc, id asc) order, a strict order: each thread keeps the best
  // promote_max of its own range, and the best of those are the best of all.
  const double theta = T.theta;
  const int64_t pmax = T.promote_max;
  auto keep_best = [&](int t) {
    auto& v = tcand[t];
    v.erase(std::remove_if(v.begin(), v.end(),
                           [&](const std::pair<double, int32_t>& c) { return !(c.first > theta); }),
            v.end());
    if ((int64_t)v.size() > pmax) {
      std::nth_element(v.begin(), v.begin() + pmax, v.end(), better);
      v.resize(pmax);
    }
  };
  if (nthr == 1) {
    keep_best(0);
  } else {
    std::vector<std::thread> pool;
    for (int t = 1; t < nthr; ++t) pool.emplace_back(keep_best, t);
    keep_best(0);
    for (auto& th : pool) th.join();
  }
  for (int t = 0; t < nthr; ++t) cand.insert(cand.end(), tcand[t].begin(), tcand[t].end());
  if ((int64_t)cand.size() > pmax) {
    std::nth_element(cand.begin(), cand.begin() + pmax, cand.end(), better);
    cand.resize(pmax);
  }
  std::sort(cand.begin(), cand.end(), better);
  ix->st.place_walk_ms = ms_since(tp);
  tp = clk::now();
  std::vector<int32_t> place;
  svf::WavpSweep& sw = T.sweep;
  for (const auto& c : cand) {
    const int32_t x = c.second;
    const int64_t slot = T.take_slot();
    if (slot >= 0) {
      T.occupy(slot, x);
      place.insert(place.end(), {(int32_t)slot, x, -1});
      continue;
    }
    if (T.C == 0) break;
    if (!sw.active()) {     // the cache is full and stays full for the rest of the batch
      const int nt = (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency()));
      // A deletion releases the vertex's slot at once, except while serving,
      // where deleted residents stay until evicted: until then every
      // resident is alive and the scattered alive bits need not be read.
      const bool check_alive = T.dead_residents;
      sw.begin(T.C, [&](int64_t s_) {
        const int32_t y = T.slot_id[s_];
        const svf::TierState::FRec& f = T.sfr[s_];   // sfr, sdeg: T.fr[y], in_degree(y)
        return !check_alive || alive(y) ? T.alpha * halve_times(f.v, T.batch - f.stamp) +
                                              T.beta * T.log1p_deg(T.sdeg[s_])
                                        : -1.0;
      }, [&](int64_t s_) {
        if (check_alive) __builtin_prefetch(&bits[T.slot_id[s_] >> 5]);
      }, T.ref.data(), nt);
    }
    const int64_t s_ = sw.evict(T.clock, T.ref.data());
    const int32_t y = T.slot_id[s_];
    T.where[y] = -1;
    T.occupy(s_, x);                        // the victim's bit was clear
    sw.place(s_, c.first);
    place.insert(place.end(), {(int32_t)s_, x, y});
    ++T.evictions;
  }
  sw.end();
  T.promotions += place.size() / 3;
  ix->st.place_evict_ms = ms_since(tp);
  tp = clk::now();
  rc = tier_apply(ix, place, st);
  ix->st.place_apply_ms = ms_since(tp);
  return rc;
}

// Cold start (Sec. 4.4): fill the cache with the highest in-degree alive
// vectors (ties by id), in that order.
int tier_warmup(svf_index* ix, hipStream_t st) {
  svf::TierState& T = ix->tier;
  int rc = tier_refresh_indegree(ix, st);
  if (rc) return rc;
  const int64_t n = ix->n_slots;
  std::vector<uint32_t> bits((n + 31) / 32 + 1, 0u);
  CK(hipMemcpyAsync(bits.data(), ix->alive, ((n + 31) / 32) * 4, hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  std::vector<int32_t> order;
  order.reserve(n);
  for (int64_t i = 0; i < n; ++i)
    if ((bits[i >> 5] >> (i & 31)) & 1u) order.push_back((int32_t)i);
  const int64_t take = std::min<int64_t>(T.free_count(), (int64_t)order.size());
  auto first = [&](int32_t a, int32_t b) {
    return T.in_degree(a) > T.in_degree(b) || (T.in_degree(a) == T.in_degree(b) && a < b);
  };
  if (take < (int64_t)order.size()) std::nth_element(order.begin(), order.begin() + take, order.end(), first);
  std::sort(order.begin(), order.begin() + take, first);
  std::vector<int32_t> place;
  for (int64_t i = 0; i < take; ++i) {
    const int32_t x = order[i];
    if (T.where[x] >= 0) continue;
    const int64_t slot = T.take_slot();
    T.occupy(slot, x);
    place.insert(place.end(), {(int32_t)slot, x, -1});
  }
  T.promotions += place.size() / 3;
  return tier_apply(ix, place, st);
}

int tier_enable(svf_index* ix, double bytes) {
  svf::TierState& T = ix->tier;
  bg_join(ix);                              // the FP32 store moves below
  const int64_t C = (int64_t)(bytes / (double)(ix->stride * 4));
  if (C < 1) return fail(SVF_E_INVAL, "cache_bytes below one vector");
  if (T.on) return fail(SVF_E_INVAL, "cache already configured");
  CK(hipMalloc(&T.cache, C * ix->stride * 4));
  T.C = C;
  T.slot_id.assign(C, -1);
  T.sfr.assign(C, svf::TierState::FRec{});
  T.dead_residents = false;
  if (T.sdeg_h.ensure(C * 4) == hipSuccess) {
    T.sdeg = T.sdeg_h.as<int32_t>();
  } else {                                  // past the host's pinning limit
    (void)hipGetLastError();
    T.sdeg_v.assign(C, 0);
    T.sdeg = T.sdeg_v.data();
  }
  std::fill(T.sdeg, T.sdeg + C, 0);
  T.ref.assign(C, 0);
  T.free_slots.clear();
  T.e_in_valid = false;
  T.used = 0;
  T.clock = 0;
  T.seg_shift = host_seg_shift(ix);
  if (ix->n_slots == 0) {
    if (ix->vec32) (void)hipFree(ix->vec32);
    ix->vec32 = nullptr;
    T.on = true;
    const int64_t cap = ix->cap;
    ix->cap = 0;                      // re-create the stores in their tiered form
    return reserve(ix, std::max<int64_t>(cap, 1024));
  }
  // a filled index: its FP32 store moves to pinned host segments, then the
  // cache is warmed with the highest in-degree vectors
  int32_t* map = nullptr;
  hipError_t e = hipSuccess;
  int rc = tier_grow_host(ix, ix->cap);
  if (rc == SVF_OK) {
    const int64_t S = int64_t(1) << T.seg_shift;
    for (size_t i = 0; i < T.seg.size() && e == hipSuccess; ++i) {
      const int64_t rows = std::min<int64_t>(T.seg_alloc[i], ix->cap - (int64_t)i * S);
      e = hipMemcpyAsync(T.seg[i], ix->vec32 + (int64_t)i * S * ix->stride,
                         (size_t)(rows * ix->stride * 4), hipMemcpyDeviceToHost, ix->stream);
    }
    if (e == hipSuccess && (e = hipMalloc(&map, ix->cap * 4)) == hipSuccess &&
        (e = svf::launch_fill_u32(map, ix->cap, 0xffffffffu, ix->stream)) == hipSuccess)
      e = hipStreamSynchronize(ix->stream);
    if (e != hipSuccess) rc = hip_fail(e, "tiered store setup");
  }
  if (rc) {
    for (float* p : T.seg) (void)hipHostFree(p);
    T.seg.clear();
    T.seg_alloc.clear();
    if (map) (void)hipFree(map);
    (void)hipFree(T.cache);
    T.cache = nullptr;
    T.C = 0;
    return rc;
  }
  (void)hipFree(ix->vec32);
  ix->vec32 = nullptr;
  T.map = map;
  T.where.assign(ix->cap, -1);
  T.fr.assign(ix->cap, svf::TierState::FRec{});
  T.freq.assign(ix->cap, 0);
  T.last.assign(ix->cap, -1);
  T.on = true;
  return tier_warmup(ix, ix->stream);
}

}  // namespace svf_detail

using namespace svf_detail;

// ===========================================================================
extern "C" {

const char* svf_last_error(void) { return g_err.c_str(); }

int svf_create(int32_t dim, int32_t degree, int32_t metric, svf_index** out) {
  if (!out) return fail(SVF_E_INVAL, "null output handle");
  *out = nullptr;
  if (dim < 1 || dim > 1024) return fail(SVF_E_INVAL, "dim must be in [1, 1024]");
  if (degree < 1 || degree > 128) return fail(SVF_E_INVAL, "degree must be in [1, 128]");
  if (metric != SVF_METRIC_L2 && metric != SVF_METRIC_IP) return fail(SVF_E_INVAL, "unknown metric");
  svf_index* ix = new (std::nothrow) svf_index();
  if (!ix) return fail(SVF_E_NOMEM, "host allocation");
  ix->dim = dim;
  ix->R = degree;
  ix->metric = metric;
  ix->stride = round_up(dim, 8);
  hipError_t e;
  if ((e = hipGetDevice(&ix->device)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&ix->stream, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipEventCreate(&ix->ev0)) != hipSuccess || (e = hipEventCreate(&ix->ev1)) != hipSuccess ||
      // both events start recorded, so timings read before any work are 0
      (e = hipEventRecord(ix->ev0, ix->stream)) != hipSuccess ||
      (e = hipEventRecord(ix->ev1, ix->stream)) != hipSuccess) {
    delete ix;
    return hip_fail(e, "device setup");
  }
  int rc = reserve(ix, 1024);
  if (rc) {
    svf_destroy(ix);
    return rc;
  }
  *out = ix;
  return SVF_OK;
}

int svf_destroy(svf_index* ix) {
  if (!ix) return SVF_OK;
  if (ix->server) serve_shutdown(ix);
  {
    std::lock_guard<std::mutex> g(ix->mu);
    bg_join(ix);
    if (ix->bg.st) (void)hipStreamDestroy(ix->bg.st);
    ix->bg.st = nullptr;
    if (ix->stream) (void)hipStreamSynchronize(ix->stream);
    if (ix->vec32) (void)hipFree(ix->vec32);
    for (float* p : ix->tier.seg) (void)hipHostFree(p);
    if (ix->veclp) (void)hipFree(ix->veclp);
    if (ix->graph) (void)hipFree(ix->graph);
    if (ix->nscale) (void)hipFree(ix->nscale);
    if (ix->edge_d) (void)hipFree(ix->edge_d);
    if (ix->alive) (void)hipFree(ix->alive);
    if (ix->tier.cache) (void)hipFree(ix->tier.cache);
    if (ix->tier.map) (void)hipFree(ix->tier.map);
    if (ix->ev0) (void)hipEventDestroy(ix->ev0);
    if (ix->ev1) (void)hipEventDestroy(ix->ev1);
    if (ix->stream) (void)hipStreamDestroy(ix->stream);
    delete ix->model;
    ix->model = nullptr;
  }
  delete ix;
  return SVF_OK;
}

int svf_set_option(svf_index* ix, const char* key, double v) {
  if (!ix || !key) return fail(SVF_E_INVAL, "null argument");
  std::lock_guard<std::mutex> g(ix->mu);
  auto is_int = [](double x) { return std::floor(x) == x; };
  std::string k(key);
  svf::Options& o = ix->opt;
  if (!std::isfinite(v)) return fail(SVF_E_INVAL, "option value must be finite");
  if (k == "seed") {
    if (v < 0 || !is_int(v)) return fail(SVF_E_INVAL, "seed must be a non-negative integer");
    o.seed = (uint64_t)v;
  } else if (k == "beam_insert") {
    if (!is_int(v) || v < ix->R || v > kMaxBeam) return fail(SVF_E_INVAL, "beam_insert in [degree, 512]");
    o.beam_insert = (int)v;
  } else if (k == "coop_max_batch") {
    if (!is_int(v) || v < 0 || v > (1 << 22)) return fail(SVF_E_INVAL, "coop_max_batch in [0, 2^22]");
    o.coop_max_batch = (int)v;
  } else if (k == "entry_samples") {
    if (!is_int(v) || v < 0 || v > kMaxEntries) return fail(SVF_E_INVAL, "entry_samples in [0, 1024]");
    o.entry_samples = (int)v;
  } else if (k == "search_width") {
    if (!is_int(v) || v < 1 || v > 4) return fail(SVF_E_INVAL, "search_width in [1, 4]");
    o.search_width = (int)v;
  } else if (k == "max_iters") {
    if (!is_int(v) || v < 0 || v > 1e9) return fail(SVF_E_INVAL, "max_iters >= 0");
    o.max_iters = (int)v;
  } else if (k == "visited_slots") {
    int t = (int)v;
    if (!is_int(v) || (t != 0 && (t < 256 || t > 16384 || (t & (t - 1)))))
      return fail(SVF_E_INVAL, "visited_slots: 0 or a power of two in [256, 16384]");
    o.visited_slots = t;
  } else if (k == "visited_compact") {
    if (v != 0 && v != 1) return fail(SVF_E_INVAL, "visited_compact 0 or 1");
    o.visited_compact = (int)v;
  } else if (k == "repair_c") {
    if (!is_int(v) || v < 1 || v > 16 || v > ix->R) return fail(SVF_E_INVAL, "repair_c in [1, min(16, degree)]");
    o.repair_c = (int)v;
  } else if (k == "prune_cap") {
    if (!is_int(v) || (v != 0 && (v < ix->R || v > 1024))) return fail(SVF_E_INVAL, "prune_cap 0 or in [degree, 1024]");
    o.prune_cap = (int)v;
  } else if (k == "consolidate_frac") {
    if (v < 0 || v > 1) return fail(SVF_E_INVAL, "consolidate_frac in [0, 1]");
    o.consolidate_frac = v;
  } else if (k == "localized_repair") {
    if (v != 0 && v != 1) return fail(SVF_E_INVAL, "localized_repair 0 or 1");
    o.localized_repair = (int)v;
  } else if (k == "consolidate_async") {
    if (v != 0 && v != 1) return fail(SVF_E_INVAL, "consolidate_async 0 or 1");
    o.consolidate_async = (int)v;
  } else if (k == "insert_batch_max") {
    if (!is_int(v) || v < 1 || v > (1 << 20)) return fail(SVF_E_INVAL, "insert_batch_max in [1, 2^20]");
    o.insert_batch_max = (int)v;
  } else if (ix->server && (k == "precision" || k == "use_model" || k == "capacity" ||
                            k == "cache_bytes")) {
    return fail(SVF_E_BUSY, "option cannot change while serving");
  } else if (k == "capacity") {
    if (!is_int(v) || v < 1 || v > (double)INT32_MAX - 64)
      return fail(SVF_E_INVAL, "capacity in [1, 2^31 - 65]");
    return reserve(ix, (int64_t)v);
  } else if (k == "cache_bytes") {
    if (v <= 0) return fail(SVF_E_INVAL, "cache_bytes > 0");
    return tier_enable(ix, v);
  } else if (k == "cache_theta") {
    if (v < 0) return fail(SVF_E_INVAL, "cache_theta >= 0");
    ix->tier.theta = v;
    ix->tier.theta0 = v;
    ix->tier.have_prev = false;
  } else if (k == "cache_theta_adapt") {
    if (v != 0 && !(v > 1 && v <= 16)) return fail(SVF_E_INVAL, "cache_theta_adapt 0 or in (1, 16]");
    ix->tier.adapt = v;
    ix->tier.have_prev = false;
  } else if (k == "cache_alpha_ratio") {
    if (v < 0 || v > 1) return fail(SVF_E_INVAL, "cache_alpha_ratio in [0, 1]");
    ix->tier.alpha = v;
    ix->tier.beta = 1.0 - v;
  } else if (k == "cache_promote_max") {
    if (!is_int(v) || v < 0 || v > (1 << 24)) return fail(SVF_E_INVAL, "cache_promote_max in [0, 2^24]");
    ix->tier.promote_max = (int)v;
  } else if (k == "cache_indegree_verify") {
    if (v != 0 && v != 1) return fail(SVF_E_INVAL, "cache_indegree_verify 0 or 1");
    ix->tier.verify_indegree = (int)v;
  } else if (k == "cache_policy") {
    if (!is_int(v) || v < 0 || v > 3) return fail(SVF_E_INVAL, "cache_policy 0 (WAVP), 1 (LRU), 2 (LFU) or 3 (LRFU)");
    ix->tier.policy = (int)v;
  } else if (k == "cache_trace_cap") {
    if (!is_int(v) || v < 16 || v > 8192) return fail(SVF_E_INVAL, "cache_trace_cap in [16, 8192]");
    ix->tier.trace_cap = (int)v;
  } else if (k == "fp8_row_scales") {
    if (v != -1 && v != 0 && v != 1) return fail(SVF_E_INVAL, "fp8_row_scales -1, 0 or 1");
    bg_join(ix);                              // its searches may read the scales freed below
    o.fp8_row_scales = (int)v;
    const int rc = row_scales_sync(ix, ix->stream);
    if (rc) return rc;
    CK(hipStreamSynchronize(ix->stream));
  } else if (k == "host_segment_rows") {
    if (ix->tier.on) return fail(SVF_E_BUSY, "host_segment_rows is set before cache_bytes");
    // (the seed rows, at most 4 * degree <= 512, sit in the first segment)
    if (v != 0 && (!is_int(v) || v < 1024 || v > (double)(1 << 30) ||
                   ((int64_t)v & ((int64_t)v - 1)) != 0))
      return fail(SVF_E_INVAL, "host_segment_rows 0 or a power of two in [1024, 2^30]");
    ix->tier.seg_rows_opt = (int64_t)v;
  } else if (k == "precision") {
    if (v != 0 && v != 1 && v != 2 && v != 3)
      return fail(SVF_E_INVAL, "precision 0 (FP32), 1 (FP16), 2 (BF16) or 3 (FP8)");
    o.precision = (int)v;
    return sync_lowp(ix);
  } else if (k == "rerank") {
    if (v != 0 && v != 1) return fail(SVF_E_INVAL, "rerank 0 or 1");
    o.rerank = (int)v;
  } else if (k == "use_model") {
    if (v != 0 && v != 1) return fail(SVF_E_INVAL, "use_model 0 or 1");
    if (v == 1 && !ix->model) return fail(SVF_E_INVAL, "use_model needs svf_model_fit first");
    o.use_model = (int)v;
  } else if (k == "model_conf") {
    if (v < 0 || v > 1) return fail(SVF_E_INVAL, "model_conf in [0, 1]");
    o.model_conf = v;
  } else if (k == "model_stop_scale") {
    if (v <= 0 || v > 1e6) return fail(SVF_E_INVAL, "model_stop_scale > 0");
    o.model_stop_scale = v;
  } else if (k == "cache_cpu_miss") {
    if (v != 0 && v != 1) return fail(SVF_E_INVAL, "cache_cpu_miss 0 or 1");
    o.cache_cpu_miss = (int)v;
  } else if (k == "model_entries") {
    if (v != 0 && v != 1) return fail(SVF_E_INVAL, "model_entries 0 or 1");
    o.model_entries = (int)v;
  } else if (k == "model_min_iters") {
    if (!is_int(v) || v < 1 || v > 1e9) return fail(SVF_E_INVAL, "model_min_iters >= 1");
    o.model_min_iters = (int)v;
  } else {
    return fail(SVF_E_INVAL, "unknown option " + k);
  }
  return SVF_OK;
}

int svf_get_option(const svf_index* ix, const char* key, double* out) {
  if (!ix || !key || !out) return fail(SVF_E_INVAL, "null argument");
  std::string k(key);
  const svf::Options& o = ix->opt;
  if (k == "seed") *out = (double)o.seed;
  else if (k == "dim") *out = ix->dim;
  else if (k == "degree") *out = ix->R;
  else if (k == "metric") *out = ix->metric;
  else if (k == "capacity") *out = (double)ix->cap;
  else if (k == "cache_resident")
    *out = (double)(ix->tier.used - (int64_t)ix->tier.free_slots.size());
  else if (k == "beam_insert") *out = beam_insert(ix);
  else if (k == "entry_samples") *out = o.entry_samples;
  else if (k == "coop_max_batch") *out = o.coop_max_batch;
  else if (k == "max_iters") *out = o.max_iters;
  else if (k == "search_width") *out = o.search_width;
  else if (k == "visited_slots") *out = o.visited_slots;
  else if (k == "visited_compact") *out = o.visited_compact;
  else if (k == "repair_c") *out = o.repair_c;
  else if (k == "prune_cap") *out = o.prune_cap;
  else if (k == "consolidate_frac") *out = o.consolidate_frac;
  else if (k == "localized_repair") *out = o.localized_repair;
  else if (k == "consolidate_async") *out = o.consolidate_async;
  else if (k == "consolidate_pending") *out = ix->bg.active ? 1.0 : 0.0;
  else if (k == "insert_batch_max") *out = o.insert_batch_max;
  else if (k == "precision") *out = o.precision;
  else if (k == "rerank") *out = o.rerank;
  else if (k == "use_model") *out = o.use_model;
  else if (k == "cache_bytes") *out = (double)(ix->tier.C * ix->stride * 4);
  else if (k == "cache_theta") *out = ix->tier.theta;
  else if (k == "cache_theta_adapt") *out = ix->tier.adapt;
  else if (k == "cache_alpha_ratio") *out = ix->tier.alpha;
  else if (k == "cache_promote_max") *out = ix->tier.promote_max;
  else if (k == "cache_trace_cap") *out = ix->tier.trace_cap;
  else if (k == "cache_policy") *out = ix->tier.policy;
  else if (k == "cache_indegree_verify") *out = ix->tier.verify_indegree;
  else if (k == "host_segment_rows")
    *out = ix->tier.on ? (double)(int64_t(1) << ix->tier.seg_shift) : (double)ix->tier.seg_rows_opt;
  else if (k == "host_segments") *out = (double)ix->tier.seg.size();
  else if (k == "fp8_row_scales") *out = o.fp8_row_scales;
  else if (k == "fp8_row_scales_on") *out = ix->nscale ? 1.0 : 0.0;
  else if (k == "model_conf") *out = o.model_conf;
  else if (k == "model_stop_scale") *out = o.model_stop_scale;
  else if (k == "model_min_iters") *out = o.model_min_iters;
  else if (k == "model_entries") *out = o.model_entries;
  else if (k == "cache_cpu_miss") *out = o.cache_cpu_miss;
  else if (k == "cache_cpu_rounds") *out = (double)ix->tier.co_rounds;
  else return fail(SVF_E_INVAL, "unknown option " + k);
  return SVF_OK;
}

int svf_insert_dev(svf_index* ix, const float* d_vecs, int64_t n, int32_t* d_out_ids, void* stream) {
  if (ix && ix->server) return fail(SVF_E_BUSY, "index is serving: use svf_submit_insert");
  if (!ix || (n > 0 && !d_vecs)) return fail(SVF_E_INVAL, "null argument");
  if (n < 0) return fail(SVF_E_INVAL, "n < 0");
  std::lock_guard<std::mutex> g(ix->mu);
  CK(hipStreamSynchronize((hipStream_t)stream));   // the producer of d_vecs (NULL: default stream)
  return insert_stream(ix, d_vecs, n, d_out_ids, nullptr);
}

int svf_insert(svf_index* ix, const float* vecs, int64_t n, int32_t* out_ids) {
  if (ix && ix->server) return fail(SVF_E_BUSY, "index is serving: use svf_submit_insert");
  if (!ix || (n > 0 && !vecs)) return fail(SVF_E_INVAL, "null argument");
  if (n < 0) return fail(SVF_E_INVAL, "n < 0");
  if (n == 0) return SVF_OK;
  if (!all_finite(vecs, n * ix->dim)) return fail(SVF_E_INVAL, "non-finite vector value");
  std::lock_guard<std::mutex> g(ix->mu);
  float* d;
  int rc = scratch_grow(ix->s_q, (size_t)n * ix->dim, &d);
  if (rc) return rc;
  CK(hipMemcpyAsync(d, vecs, (size_t)n * ix->dim * 4, hipMemcpyHostToDevice, ix->stream));
  return insert_stream(ix, d, n, nullptr, out_ids);
}

int svf_build(svf_index* ix, const float* vecs, int64_t n) {
  if (ix && ix->server) return fail(SVF_E_BUSY, "index is serving: stop serving first");
  if (!ix || (n > 0 && !vecs)) return fail(SVF_E_INVAL, "null argument");
  if (n < 1) return fail(SVF_E_INVAL, "n must be >= 1");
  if (ix->n_slots != 0) return fail(SVF_E_INVAL, "build needs an empty index");
  if (!all_finite(vecs, n * ix->dim)) return fail(SVF_E_INVAL, "non-finite vector value");
  std::lock_guard<std::mutex> g(ix->mu);
  int rc = reserve(ix, n);
  if (rc) return rc;
  float* d;
  if ((rc = scratch_grow(ix->s_q, (size_t)n * ix->dim, &d))) return rc;
  CK(hipMemcpyAsync(d, vecs, (size_t)n * ix->dim * 4, hipMemcpyHostToDevice, ix->stream));
  ix->tier.building = true;
  rc = insert_stream(ix, d, n, nullptr, nullptr);
  ix->tier.building = false;
  if (rc == SVF_OK && ix->tier.on) rc = tier_warmup(ix, ix->stream);
  return rc;
}

int svf_delete(svf_index* ix, const int32_t* ids, int64_t n) {
  if (!ix || (n > 0 && !ids)) return fail(SVF_E_INVAL, "null argument");
  if (n < 0) return fail(SVF_E_INVAL, "n < 0");
  if (ix->server) return fail(SVF_E_BUSY, "index is serving: use svf_submit_delete");
  std::lock_guard<std::mutex> g(ix->mu);
  return delete_ids(ix, ids, n);
}

int svf_consolidate(svf_index* ix) {
  if (ix && ix->server) return fail(SVF_E_BUSY, "index is serving: stop serving first");
  if (!ix) return fail(SVF_E_INVAL, "null index");
  std::lock_guard<std::mutex> g(ix->mu);
  int rc = bg_merge(ix);
  if (rc) return rc;
  rc = repair(ix, 1);
  ix->deleted_since = 0;
  ix->alive_at_consolidate = ix->n_alive;
  return rc;
}

int svf_consolidate_wait(svf_index* ix) {
  if (ix && ix->server) return fail(SVF_E_BUSY, "index is serving: the serving loop merges");
  if (!ix) return fail(SVF_E_INVAL, "null index");
  std::lock_guard<std::mutex> g(ix->mu);
  return bg_merge(ix);
}

int svf_search_dev(svf_index* ix, const float* d_queries, int64_t nq, int32_t k, int32_t beam,
                   int32_t* d_out_ids, float* d_out_dists, int32_t* d_n_dist, int32_t* d_n_exp,
                   void* stream) {
  if (ix && ix->server) return fail(SVF_E_BUSY, "index is serving: use svf_submit_search");
  int rc = check_search_args(ix, nq, k, beam);
  if (rc) return rc;
  if (nq > 0 && (!d_queries || !d_out_ids || !d_out_dists)) return fail(SVF_E_INVAL, "null buffer");
  std::lock_guard<std::mutex> g(ix->mu);
  hipStream_t st = (hipStream_t)stream;        // NULL is the default stream
  rc = search_impl(ix, d_queries, nq, k, beam, d_out_ids, d_out_dists, d_n_dist, d_n_exp, st);
  if (rc == SVF_OK && ix->tier.on && ix->n_slots > 0 && nq > 0) rc = tier_after_batch(ix, nq, st);
  return rc;
}

int svf_search(svf_index* ix, const float* queries, int64_t nq, int32_t k, int32_t beam,
               int32_t* out_ids, float* out_dists) {
  if (ix && ix->server) return fail(SVF_E_BUSY, "index is serving: use svf_submit_search");
  int rc = check_search_args(ix, nq, k, beam);
  if (rc) return rc;
  if (nq == 0) return SVF_OK;
  if (!queries || !out_ids || !out_dists) return fail(SVF_E_INVAL, "null buffer");
  if (!all_finite(queries, nq * ix->dim)) return fail(SVF_E_INVAL, "non-finite query value");
  std::lock_guard<std::mutex> g(ix->mu);
  hipStream_t st = ix->stream;
  float *dq, *dd;
  int32_t* di;
  if ((rc = scratch_grow(ix->s_q, (size_t)nq * ix->dim, &dq)) || (rc = scratch_grow(ix->s_ids, (size_t)nq * k, &di)) ||
      (rc = scratch_grow(ix->s_d, (size_t)nq * k, &dd)))
    return rc;
  CK(hipMemcpyAsync(dq, queries, (size_t)nq * ix->dim * 4, hipMemcpyHostToDevice, st));
  rc = search_impl(ix, dq, nq, k, beam, di, dd, nullptr, nullptr, st);
  if (rc) return rc;
  CK(hipMemcpyAsync(out_ids, di, (size_t)nq * k * 4, hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(out_dists, dd, (size_t)nq * k * 4, hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  finish_search_stats(ix);
  if (ix->tier.on && ix->n_slots > 0) return tier_after_batch(ix, nq, st);
  return SVF_OK;
}

int svf_search_listed(svf_index* ix, const float* queries, int64_t nq, int32_t k, int32_t beam,
                      const int32_t* entries, int32_t ecap, const int32_t* max_iters,
                      int32_t* out_ids, float* out_dists) {
  if (ix && ix->server) return fail(SVF_E_BUSY, "index is serving: stop serving first");
  int rc = check_search_args(ix, nq, k, beam);
  if (rc) return rc;
  if (nq == 0) return SVF_OK;
  if (!queries || !entries || !out_ids || !out_dists || ecap < 1) return fail(SVF_E_INVAL, "bad buffer");
  if (!all_finite(queries, nq * ix->dim)) return fail(SVF_E_INVAL, "non-finite query value");
  std::lock_guard<std::mutex> g(ix->mu);
  hipStream_t st = ix->stream;
  float *dq, *dd;
  int32_t *di, *de, *dqe, *dqm;
  uint64_t* qkey;
  if ((rc = scratch_grow(ix->s_q, (size_t)nq * ix->dim, &dq)) || (rc = scratch_grow(ix->s_ids, (size_t)nq * k, &di)) ||
      (rc = scratch_grow(ix->s_d, (size_t)nq * k, &dd)) || (rc = scratch_grow(ix->s_misc[0], (size_t)nq * ecap, &de)) ||
      (rc = scratch_grow(ix->s_misc[1], nq, &dqe)) || (rc = scratch_grow(ix->s_misc[2], nq, &dqm)) ||
      (rc = scratch_grow(ix->s_qkey, nq, &qkey)))
    return rc;
  std::vector<int32_t> qe(nq), qm(nq, 0);
  for (int64_t i = 0; i < nq; ++i) {
    qe[i] = (int32_t)i;
    if (max_iters) qm[i] = max_iters[i];
  }
  CK(hipMemcpyAsync(dq, queries, (size_t)nq * ix->dim * 4, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(de, entries, (size_t)nq * ecap * 4, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dqe, qe.data(), (size_t)nq * 4, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dqm, qm.data(), (size_t)nq * 4, hipMemcpyHostToDevice, st));
  if (ix->n_slots == 0) {
    CK(svf::launch_fill_u32(di, nq * k, 0xffffffffu, st));
    CK(svf::launch_fill_u32(dd, nq * k, 0x7f800000u, st));
  } else {
    svf::SearchArgs a = base_args(ix);
    set_beam(a, ix, beam);
    a.k = k;
    a.queries = dq;
    a.qstride = ix->dim;
    a.nq = (int)nq;
    a.entry_lists = de;
    a.entry_cap = ecap;
    a.q_entry = dqe;
    a.q_max_iters = dqm;
    a.out_ids = di;
    a.out_d = dd;
    CK(svf::launch_query_keys(dq, ix->dim, nullptr, ix->dim, a.nq, ix->opt.seed, qkey, st));
    a.qkey = qkey;
    CK(svf::launch_search(a, ix->veclp_prec, st));
  }
  CK(hipMemcpyAsync(out_ids, di, (size_t)nq * k * 4, hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(out_dists, dd, (size_t)nq * k * 4, hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  return SVF_OK;
}

int svf_search_trace(svf_index* ix, const float* queries, int64_t nq, int32_t k, int32_t beam,
                     int32_t* out_ids, float* out_dists, int32_t* out_last_change) {
  if (ix && ix->server) return fail(SVF_E_BUSY, "index is serving: stop serving first");
  int rc = check_search_args(ix, nq, k, beam);
  if (rc) return rc;
  if (nq == 0) return SVF_OK;
  if (!queries || !out_ids || !out_dists || !out_last_change) return fail(SVF_E_INVAL, "null buffer");
  if (!all_finite(queries, nq * ix->dim)) return fail(SVF_E_INVAL, "non-finite query value");
  std::lock_guard<std::mutex> g(ix->mu);
  hipStream_t st = ix->stream;
  float *dq, *dd;
  int32_t *di, *dl;
  uint64_t* qkey;
  if ((rc = scratch_grow(ix->s_q, (size_t)nq * ix->dim, &dq)) || (rc = scratch_grow(ix->s_ids, (size_t)nq * k, &di)) ||
      (rc = scratch_grow(ix->s_d, (size_t)nq * k, &dd)) || (rc = scratch_grow(ix->s_misc[1], nq, &dl)) ||
      (rc = scratch_grow(ix->s_qkey, nq, &qkey)))
    return rc;
  CK(hipMemcpyAsync(dq, queries, (size_t)nq * ix->dim * 4, hipMemcpyHostToDevice, st));
  if (ix->n_slots == 0) {
    CK(svf::launch_fill_u32(di, nq * k, 0xffffffffu, st));
    CK(svf::launch_fill_u32(dd, nq * k, 0x7f800000u, st));
    CK(svf::launch_fill_u32(dl, nq, 0u, st));
  } else {
    svf::SearchArgs a = base_args(ix);
    set_beam(a, ix, beam);
    a.k = k;
    a.queries = dq;
    a.qstride = ix->dim;
    a.nq = (int)nq;
    a.out_ids = di;
    a.out_d = dd;
    a.last_change = dl;
    CK(svf::launch_query_keys(dq, ix->dim, nullptr, ix->dim, a.nq, ix->opt.seed, qkey, st));
    a.qkey = qkey;
    CK(svf::launch_search(a, ix->veclp_prec, st));
  }
  CK(hipMemcpyAsync(out_ids, di, (size_t)nq * k * 4, hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(out_dists, dd, (size_t)nq * k * 4, hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(out_last_change, dl, (size_t)nq * 4, hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  return SVF_OK;
}

int svf_model_get(const svf_index* cix, int32_t* n_clusters, int32_t* entry_cap, float* params,
                  int64_t params_cap, int32_t* entry_lists, int64_t lists_cap) {
  if (!cix) return fail(SVF_E_INVAL, "null index");
  svf_index* ix = const_cast<svf_index*>(cix);
  std::lock_guard<std::mutex> g(ix->mu);
  if (!ix->model) return fail(SVF_E_NOTFOUND, "no trained predictor: call svf_model_fit first");
  const svf::MlpDims& d = ix->model->dims();
  if (n_clusters) *n_clusters = ix->model_nc;
  if (entry_cap) *entry_cap = ix->entry_cap;
  if (params) {
    if (params_cap < d.total()) return fail(SVF_E_INVAL, "params_cap below the parameter count");
    CK(hipStreamSynchronize(ix->stream));
    CK(ix->model->get_params(params, ix->stream));
    // the forward pass multiplies by the weights rounded to BF16 (nearest even)
    auto rnd = [](float& x) {
      uint32_t u;
      std::memcpy(&u, &x, 4);
      u += 0x7fffu + ((u >> 16) & 1u);
      u &= 0xffff0000u;
      std::memcpy(&x, &u, 4);
    };
    for (int64_t i = d.o_w1(); i < d.o_b1(); ++i) rnd(params[i]);
    for (int64_t i = d.o_w2(); i < d.o_b2(); ++i) rnd(params[i]);
    for (int64_t i = d.o_w3(); i < d.o_b3(); ++i) rnd(params[i]);
  }
  if (entry_lists) {
    const int64_t n = (int64_t)ix->model_nc * ix->entry_cap;
    if (lists_cap < n) return fail(SVF_E_INVAL, "lists_cap below n_clusters * entry_cap");
    CK(hipStreamSynchronize(ix->stream));
    CK(hipMemcpy(entry_lists, ix->entry_lists.as<int32_t>(), n * 4, hipMemcpyDeviceToHost));
  }
  return SVF_OK;
}

int svf_model_fit(svf_index* ix, const float* train_queries, int64_t n, int32_t k, int32_t beam,
                  int32_t n_clusters, int32_t epochs, float* last_loss) {
  if (ix && ix->server) return fail(SVF_E_BUSY, "index is serving: stop serving first");
  int rc = check_search_args(ix, n, k, beam);
  if (rc) return rc;
  if (!train_queries || n < 1024) return fail(SVF_E_INVAL, "need at least 1024 training queries");
  if (n_clusters < 2 || n_clusters > 256) return fail(SVF_E_INVAL, "n_clusters in [2, 256]");
  if (epochs < 1 || epochs > 1000) return fail(SVF_E_INVAL, "epochs in [1, 1000]");
  if (!all_finite(train_queries, n * ix->dim)) return fail(SVF_E_INVAL, "non-finite query value");
  std::lock_guard<std::mutex> g(ix->mu);
  if (ix->tier.on)
    return fail(SVF_E_INVAL, "the predictor is fitted on an index whose FP32 store is in HBM "
                             "(not with cache_bytes)");
  if (ix->n_alive < 2 * n_clusters) return fail(SVF_E_INVAL, "index too small for the clusters");
  hipStream_t st = ix->stream;
  const int dim = ix->dim, nc = n_clusters, ecap = 64;
  // 1. entry clusters: Lloyd k-means over an evenly spaced sample of rows
  const int64_t ns = std::min<int64_t>(ix->n_slots, 65536);
  const int64_t step = ix->n_slots / ns;
  float* cent;
  int32_t* sassign;
  if ((rc = scratch(ix->centroids, (size_t)nc * dim, &cent)) ||
      (rc = scratch(ix->s_misc[0], ns, &sassign)))
    return rc;
  CK(hipMemcpy2DAsync(cent, dim * 4, ix->vec32, step * ix->stride * 4, dim * 4, nc,
                      hipMemcpyDeviceToDevice, st));
  CK(svf::kmeans(ix->vec32, ns, step * ix->stride, dim, nc, 12, cent, sassign, st));
  // 2. traces of plain search: top-k ids and the step where the top-k settled
  float* dq;
  int32_t *ids, *lcg, *labels;
  float *dd, *lstop;
  uint64_t* qkey;
  if ((rc = scratch(ix->s_q, (size_t)n * dim, &dq)) || (rc = scratch(ix->s_ids, (size_t)n * k, &ids)) ||
      (rc = scratch(ix->s_d, (size_t)n * k, &dd)) || (rc = scratch(ix->s_misc[1], n, &lcg)) ||
      (rc = scratch(ix->s_misc[2], n, &labels)) || (rc = scratch(ix->s_misc[3], n, &lstop)) ||
      (rc = scratch(ix->s_qkey, n, &qkey)))
    return rc;
  CK(hipMemcpyAsync(dq, train_queries, (size_t)n * dim * 4, hipMemcpyHostToDevice, st));
  svf::SearchArgs a = base_args(ix);
  set_beam(a, ix, beam);
  a.k = k;
  a.queries = dq;
  a.qstride = dim;
  a.nq = (int)n;
  a.out_ids = ids;
  a.out_d = dd;
  a.last_change = lcg;
  CK(svf::launch_query_keys(dq, dim, nullptr, dim, a.nq, ix->opt.seed, qkey, st));
  a.qkey = qkey;
  CK(svf::launch_search(a, ix->veclp_prec, st));
  // 3. labels: cluster of the top-1 result; log of the settling step
  CK(svf::assign_rows(ix->vec32, ix->stride, dim, ids, n, k, cent, nc, labels, st));
  CK(svf::launch_log_steps(lcg, n, lstop, st));
  CK(hipStreamSynchronize(st));
  // 4. per-cluster entry lists: spread over the cluster, or nearest to its centroid
  int32_t* el;
  float* eld;
  uint64_t* ckey;
  if ((rc = scratch(ix->entry_lists, (size_t)nc * ecap, &el)) ||
      (rc = scratch(ix->s_misc[4], (size_t)nc * ecap, &eld)) || (rc = scratch(ix->s_misc[5], nc, &ckey)))
    return rc;
  if (ix->opt.model_entries == 1) {
    CK(svf::launch_spread_entries(sassign, ns, step, ix->alive, nc, ecap, el, st));
  } else {
    svf::SearchArgs c = base_args(ix);
    set_beam(c, ix, std::max(2 * ecap, beam));
    c.k = ecap;
    c.queries = cent;
    c.qstride = dim;
    c.nq = nc;
    c.out_ids = el;
    c.out_d = eld;
    CK(svf::launch_query_keys(cent, dim, nullptr, dim, nc, ix->opt.seed, ckey, st));
    c.qkey = ckey;
    CK(svf::launch_search(c, ix->veclp_prec, st));
  }
  ix->entry_cap = ecap;
  // 5. train the predictor on the GPU, in two stages: first on the labels of
  //    plain search; then the stop labels are re-measured on traces of the
  //    search that starts from the predicted clusters' entry lists (the form
  //    the predictor will drive), and training continues on them
  delete ix->model;
  ix->model = new (std::nothrow) svf::Mlp(dim, 256, nc, ix->opt.seed + 12345);
  if (!ix->model) return fail(SVF_E_NOMEM, "host allocation");
  CK(ix->model->init_device(st));
  ix->model_nc = nc;
  const int e1 = std::max(1, epochs / 2), e2 = epochs - e1;
  float loss = 0.f;
  CK(ix->model->train(dq, labels, lstop, n, e1, 1024, 2e-3f, 0.1f, 1.0f, &loss, st));
  if (e2 > 0) {
    float* z;
    int32_t *qe, *qm;
    if ((rc = scratch(ix->s_z, (size_t)n * (nc + 1), &z)) || (rc = scratch(ix->s_qentry, n, &qe)) ||
        (rc = scratch(ix->s_qmax, n, &qm)))
      return rc;
    CK(ix->model->forward(dq, n, z, st));
    CK(svf::launch_model_decide(z, n, nc, 0.0f, 1.0f, 1, qe, qm, nullptr, st));
    svf::SearchArgs t = base_args(ix);
    set_beam(t, ix, beam);
    t.k = k;
    t.queries = dq;
    t.qstride = dim;
    t.nq = (int)n;
    t.out_ids = ids;
    t.out_d = dd;
    t.last_change = lcg;
    t.entry_lists = el;
    t.entry_cap = ecap;
    t.q_entry = qe;
    t.qkey = qkey;
    CK(svf::launch_search(t, ix->veclp_prec, st));
    CK(svf::launch_log_steps(lcg, n, lstop, st));
    CK(ix->model->train(dq, labels, lstop, n, e2, 1024, 1e-3f, 0.1f, 1.0f, &loss, st));
  }
  CK(hipStreamSynchronize(st));
  if (last_loss) *last_loss = loss;
  return SVF_OK;
}

int svf_stats_get(const svf_index* cix, svf_stats* out) {
  if (!cix || !out) return fail(SVF_E_INVAL, "null argument");
  svf_index* ix = const_cast<svf_index*>(cix);
  std::lock_guard<std::mutex> g(ix->mu);
  (void)hipDeviceSynchronize();
  finish_search_stats(ix);
  ix->st.n_slots = ix->n_slots;
  ix->st.n_alive = ix->n_alive;
  ix->st.capacity = ix->cap;
  ix->st.device_bytes = ix->cap * ((ix->tier.on ? 0 : ix->stride * 4) + ix->R * 8 + 8) + ix->cap / 8 +
                        (ix->veclp_prec ? (int64_t)lp_bytes(ix, ix->veclp_prec, ix->cap) : 0) +
                        ix->tier.C * ix->stride * 4 + (ix->nscale ? ix->cap * ix->R * 4 : 0);
  ix->st.cache_slots = ix->tier.C;
  ix->st.cache_gather_hits = (int64_t)ix->tier.gather_hits;
  ix->st.cache_gather_misses = (int64_t)ix->tier.gather_misses;
  ix->st.cache_last_trace_hits = ix->tier.last_trace_hits;
  ix->st.cache_last_placed = ix->tier.last_placed;
  ix->st.cache_promotions = (int64_t)ix->tier.promotions;
  ix->st.cache_evictions = (int64_t)ix->tier.evictions;
  ix->st.long_lists = ix->lrev.lists + ix->rs.lg.lists + ix->bg.rs.lg.lists;
  *out = ix->st;
  return SVF_OK;
}

int svf_export_graph(const svf_index* cix, int32_t* rows, float* edge_d, uint8_t* alive, int64_t cap_slots) {
  if (!cix) return fail(SVF_E_INVAL, "null index");
  svf_index* ix = const_cast<svf_index*>(cix);
  std::lock_guard<std::mutex> g(ix->mu);
  if (cap_slots < ix->n_slots) return fail(SVF_E_INVAL, "cap_slots < n_slots");
  const int64_t n = ix->n_slots;
  CK(hipStreamSynchronize(ix->stream));
  if (rows && n) CK(hipMemcpy(rows, ix->graph, n * ix->R * 4, hipMemcpyDeviceToHost));
  if (edge_d && n) CK(hipMemcpy(edge_d, ix->edge_d, n * ix->R * 4, hipMemcpyDeviceToHost));
  if (alive && n) {
    std::vector<uint32_t> bits((n + 31) / 32);
    CK(hipMemcpy(bits.data(), ix->alive, bits.size() * 4, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; ++i) alive[i] = (bits[i >> 5] >> (i & 31)) & 1u;
  }
  return SVF_OK;
}

int svf_cache_slots(const svf_index* cix, int32_t* slot_ids, int64_t cap, int64_t* clock) {
  if (!cix || (!slot_ids && cap > 0)) return fail(SVF_E_INVAL, "null argument");
  svf_index* ix = const_cast<svf_index*>(cix);
  std::lock_guard<std::mutex> g(ix->mu);
  const svf::TierState& T = ix->tier;
  if (cap < T.C) return fail(SVF_E_INVAL, "cap < cache slots");
  for (int64_t s = 0; s < T.C; ++s) slot_ids[s] = T.slot_id[s];
  if (clock) *clock = T.clock;
  return SVF_OK;
}

int svf_cache_calibrate(svf_index* ix, double* out) {
  if (!ix) return fail(SVF_E_INVAL, "null index");
  if (ix->server) return fail(SVF_E_BUSY, "index is serving: stop serving first");
  std::lock_guard<std::mutex> g(ix->mu);
  svf::TierState& T = ix->tier;
  if (!T.on || ix->n_slots == 0) return fail(SVF_E_INVAL, "no tiered store, or an empty index");
  std::vector<int32_t> occ;
  for (int64_t s = 0; s < T.C; ++s)
    if (T.slot_id[s] >= 0) occ.push_back((int32_t)s);
  if (occ.empty()) return fail(SVF_E_INVAL, "the cache holds no vector");
  const int ns = 65536, nx = 2048;
  std::vector<int32_t> hit(ns), miss(ns), xfer(nx);
  uint64_t z = 0x5eedULL;
  auto next = [&]() {                        // SplitMix64 (Steele, Lea and Flood, 2014)
    uint64_t r = (z += 0x9E3779B97F4A7C15ULL);
    r = (r ^ (r >> 30)) * 0xBF58476D1CE4E5B9ULL;
    r = (r ^ (r >> 27)) * 0x94D049BB133111EBULL;
    return r ^ (r >> 31);
  };
  for (int i = 0; i < ns; ++i) hit[i] = occ[next() % occ.size()];
  for (int i = 0; i < ns; ++i) miss[i] = (int32_t)(next() % (uint64_t)ix->n_slots);
  for (int i = 0; i < nx; ++i) xfer[i] = (int32_t)(next() % (uint64_t)ix->n_slots);
  svf::DevBuf ibuf, qbuf, obuf, dbuf;
  CK(ibuf.ensure((size_t)(2 * ns + nx) * 4));
  CK(qbuf.ensure((size_t)ix->stride * 4));
  CK(obuf.ensure((size_t)ns * 4));
  CK(dbuf.ensure((size_t)nx * ix->stride * 4));
  int32_t* d_hit = ibuf.as<int32_t>();
  int32_t* d_miss = d_hit + ns;
  int32_t* d_xfer = d_miss + ns;
  hipStream_t st = ix->stream;
  CK(hipMemcpyAsync(d_hit, hit.data(), ns * 4, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(d_miss, miss.data(), ns * 4, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(d_xfer, xfer.data(), nx * 4, hipMemcpyHostToDevice, st));
  CK(svf::launch_fill_u32(qbuf.as<uint32_t>(), ix->stride, 0u, st));
  // each probe: one untimed run, then the median of five timed ones
  auto timed = [&](auto&& launch, double* ms) -> int {
    CK(launch());
    std::vector<double> t;
    for (int r = 0; r < 5; ++r) {
      CK(hipEventRecord(ix->ev0, st));
      CK(launch());
      CK(hipEventRecord(ix->ev1, st));
      CK(hipEventSynchronize(ix->ev1));
      float m = 0.f;
      CK(hipEventElapsedTime(&m, ix->ev0, ix->ev1));
      t.push_back(m);
    }
    std::sort(t.begin(), t.end());
    *ms = t[2];
    return SVF_OK;
  };
  double ms_hit = 0, ms_miss = 0, ms_x = 0;
  int rc;
  if ((rc = timed([&] { return svf::launch_probe_gather(T.cache, svf::HostSegs{nullptr, 0}, d_hit,
                                                        ns, ix->stride, ix->dim, qbuf.as<float>(),
                                                        obuf.as<float>(), st); },
                  &ms_hit)) ||
      (rc = timed([&] { return svf::launch_probe_gather(nullptr, T.segs(), d_miss, ns, ix->stride,
                                                        ix->dim, qbuf.as<float>(), obuf.as<float>(),
                                                        st); },
                  &ms_miss)) ||
      (rc = timed([&] { return svf::launch_gather_rows(T.segs(), d_xfer, nx, ix->stride,
                                                       dbuf.as<float>(), st); },
                  &ms_x)))
    return rc;
  const double t_hit = ms_hit * 1e6 / ns, t_x = ms_x * 1e6 / nx;
  // the miss path in force: host-core distances (co-processing, the paper's
  // T_CPU) or reads of the host rows across the link inside the GPU gather
  const double t_miss = ix->opt.cache_cpu_miss ? host_distance_ns(ix, miss.data(), ns)
                                               : ms_miss * 1e6 / ns;
  if (!(t_miss > t_hit)) return fail(SVF_E_INTERNAL, "a host read measured no slower than a cached one");
  const double theta = t_x / (t_miss - t_hit);
  T.theta = T.theta0 = theta;
  T.have_prev = false;
  if (out) {
    out[0] = t_hit;
    out[1] = t_miss;
    out[2] = t_x;
    out[3] = theta;
  }
  return SVF_OK;
}

int svf_import_graph(svf_index* ix, const float* vecs, int64_t n, const int32_t* rows,
                     const float* edge_d, const uint8_t* alive) {
  if (ix && ix->server) return fail(SVF_E_BUSY, "index is serving: stop serving first");
  if (!ix || (n > 0 && (!vecs || !rows || !edge_d || !alive))) return fail(SVF_E_INVAL, "null argument");
  if (n < 0) return fail(SVF_E_INVAL, "n < 0");
  std::lock_guard<std::mutex> g(ix->mu);
  if (ix->n_slots != 0) return fail(SVF_E_INVAL, "import needs an empty index");
  if (!all_finite(vecs, n * ix->dim)) return fail(SVF_E_INVAL, "non-finite vector value");
  for (int64_t i = 0; i < n * ix->R; ++i)
    if (rows[i] < -1 || rows[i] >= n) return fail(SVF_E_INVAL, "row entry out of range");
  ix->tier.e_in_valid = false;
  int rc = reserve(ix, std::max<int64_t>(n, 1));
  if (rc) return rc;
  hipStream_t st = ix->stream;
  float* d;
  if ((rc = scratch_grow(ix->s_q, (size_t)std::max<int64_t>(n, 1) * ix->dim, &d))) return rc;
  CK(hipMemcpyAsync(d, vecs, n * ix->dim * 4, hipMemcpyHostToDevice, st));
  rc = store_rows(ix, d, n, 0, st);
  if (rc) return rc;
  CK(hipMemcpyAsync(ix->graph, rows, n * ix->R * 4, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(ix->edge_d, edge_d, n * ix->R * 4, hipMemcpyHostToDevice, st));
  std::vector<uint32_t> bits((n + 31) / 32 + 1, 0u);
  int64_t na = 0;
  for (int64_t i = 0; i < n; ++i)
    if (alive[i]) { bits[i >> 5] |= 1u << (i & 31); ++na; }
  CK(hipMemcpyAsync(ix->alive, bits.data(), ((n + 31) / 32) * 4, hipMemcpyHostToDevice, st));
  CK(hipStreamSynchronize(st));
  ix->n_slots = n;
  ix->n_alive = na;
  if ((rc = row_scales_sync(ix, st))) return rc;
  CK(hipStreamSynchronize(st));
  return SVF_OK;
}

}  // extern "C"
