/*
 * svf_oracle.c -- plain, slow, FP64 CPU oracle for the streaming graph-ANN
 * method of SVFusion (arXiv 2601.08528).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP library: every routine below is written out again
 * from the paper and from the published definitions it cites.
 *
 * Arithmetic: every vector value arrives as FP32 and is widened exactly to
 * double; distances, sums and comparisons are FP64.  Keys are ordered by
 * (distance, id) lexicographically everywhere, which makes every result unique.
 *
 * What follows the paper, and where:
 *   - distance: squared Euclidean (Sec. 2.1 uses the L2 norm; the square keeps
 *     the ranking) or negative inner product for the inner-product workload;
 *   - search: Algorithm 1 restricted to the device tier -- random candidate
 *     pool initialisation, repeat {nearest unexpanded, fetch its neighbours,
 *     distances, pool update} until nothing is left to expand, then the k
 *     nearest (Sec. 4.2, Algorithm 1; entry points are random, Sec. 2.3);
 *   - insertion: batched search for candidates, rank-based candidate
 *     reordering by detour counts, reverse-edge insertion (Sec. 5.1);
 *   - deletion: bitset marking, localized topology-aware repair of vertices
 *     with more than half of their neighbours deleted using at most c = 8
 *     out-neighbours of each deleted neighbour, and global consolidation past a
 *     deleted fraction of 20% (Sec. 5.2).
 * Readings of points the paper leaves open are listed beside each routine.
 *
 * Counter-based random numbers (entry points) use two published generators:
 * FNV-1a 64-bit (Fowler, Noll, Vo) over the query's bytes to derive a
 * per-query stream key, and SplitMix64 (Steele, Lea, Flood, OOPSLA 2014)
 * whose j-th output from state s is mix(s + (j+1) * golden-gamma).
 */
#include <limits.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_INVALID (-1)
enum { ORC_L2 = 0, ORC_IP = 1 };
enum { ORC_OK = 0, ORC_E_INVAL = -1, ORC_E_NOMEM = -2, ORC_E_NOTFOUND = -4 };
enum { ORC_P_FP32 = 0, ORC_P_FP16 = 1, ORC_P_BF16 = 2, ORC_P_FP8 = 3 };

typedef struct {
    int dim, R, metric;
    int64_t cap, n_slots, n_alive;
    double *vec;      /* cap x dim, exact FP32 values                       */
    double *vec_lp;   /* cap x dim, values rounded to the search precision  */
    float *vec_f32;   /* cap x dim, the FP32 input words (for hashing)      */
    int32_t *rows;    /* cap x R  neighbour ids, canonical (d,id) order     */
    double *edge_d;   /* cap x R  edge distances                            */
    uint8_t *alive;   /* cap                                                */
    uint64_t seed;
    int beam_insert;      /* candidate pool size of the insertion search     */
    int entry_samples;    /* random entry samples E (0: same as the pool)    */
    int search_width;     /* parents expanded per iteration                  */
    int max_iters;        /* 0: no cap                                       */
    int repair_c;         /* c of the localized repair                       */
    int localized_repair; /* repair affected vertices after each deletion    */
    int consolidate_async; /* consolidations run on a snapshot, merged later */
    /* a consolidation computed on a snapshot of bg_n0 vertices, staged, and
     * the forward rows of the vertices inserted since (ids bg_n0 on) */
    int bg_active;
    int64_t bg_n0;
    uint8_t *bg_changed;
    int32_t *bg_rows;
    double *bg_rows_d;
    int32_t *log_rows;
    double *log_d;
    int64_t log_n, log_cap;
    int prune_cap;        /* longest candidate list handed to the prune      */
    int precision;        /* ORC_P_*: value grid of the search distances     */
    double consolidate_frac;
    int64_t insert_batch_max; /* largest batch of one insertion pass          */
    int64_t deleted_since;  /* deletions since the last consolidation        */
    int64_t alive_at_consolidate;
} orc_index;

/* ------------------------------------------------------------------------ */
/* Rounding FP32 values to reduced-precision grids, from the IEEE-754
 * definitions: round to nearest, ties to even, on the target significand. */
static double round_to_grid(double x, int mant_bits, int min_exp, double max_finite)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(x, &e);            /* x = f * 2^e with 0.5 <= |f| < 1 */
    e -= 1;                  /* now x = g * 2^e with 1 <= |g| < 2 */
    if (e < min_exp) e = min_exp;           /* subnormal range: fixed quantum */
    double quantum = ldexp(1.0, e - mant_bits);
    double r = rint(x / quantum) * quantum; /* rint: nearest, ties to even */
    if (fabs(r) > max_finite) r = copysign(INFINITY, r);
    return r;
}
/* binary16: 10 fraction bits, emin = -14, max 65504 */
static double to_fp16(double x) { return round_to_grid(x, 10, -14, 65504.0); }
/* bfloat16: 7 fraction bits, emin = -126, max finite = (2 - 2^-7) * 2^127 */
static double to_bf16(double x) { return round_to_grid(x, 7, -126, ldexp(255.0, 120)); }

static double lp_value(int precision, float v)
{
    if (precision == ORC_P_FP16) return to_fp16((double)v);
    if (precision == ORC_P_BF16) return to_bf16((double)v);
    return (double)v;
}

/* OCP FP8 E4M3 ("E4M3FN"): 4 exponent bits with bias 7, 3 fraction bits,
 * smallest normal 2^-6, no infinities, largest finite 448.  Round to nearest,
 * ties to even; magnitudes beyond 448 saturate to 448. */
static double to_e4m3(double x)
{
    double r = round_to_grid(x, 3, -6, 448.0);
    if (isinf(r)) r = copysign(448.0, x);
    return r;
}

/* Per-vector scale of the FP8 form: the largest magnitude over 448, an FP32
 * quotient (1 for an all-zero vector), so that the largest element maps to
 * the largest finite code. */
static float fp8_scale(const float *x, int d)
{
    float m = 0.0f;
    for (int i = 0; i < d; ++i) { float a = fabsf(x[i]); if (a > m) m = a; }
    return m > 0.0f ? m / 448.0f : 1.0f;
}

/* The values a vector takes on the search grid.  FP16/BF16: each element
 * rounded.  FP8: code c_i = E4M3(x_i / s) of the FP32 quotient; a stored
 * vector is reconstructed exactly as s * c_i, a query as the FP32 product
 * s * c_i (it is held in FP32 while it searches). */
static void lp_vector(int precision, const float *x, int d, int is_query, double *out)
{
    if (precision == ORC_P_FP8) {
        const float s = fp8_scale(x, d);
        for (int i = 0; i < d; ++i) {
            const float t = x[i] / s;
            const double c = to_e4m3((double)t);
            out[i] = is_query ? (double)(s * (float)c) : (double)s * c;
        }
        return;
    }
    for (int i = 0; i < d; ++i) out[i] = lp_value(precision, x[i]);
}

/* ------------------------------------------------------------------------ */
/* Distances (Sec. 2.1): squared L2, or -<q,x> for the inner-product metric. */
static double dist(int metric, const double *a, const double *b, int dim)
{
    double s = 0.0;
    if (metric == ORC_L2) {
        for (int i = 0; i < dim; ++i) { double t = a[i] - b[i]; s += t * t; }
        return s;
    }
    for (int i = 0; i < dim; ++i) s += a[i] * b[i];
    return -s;
}

static int key_less(double da, int32_t ia, double db, int32_t ib)
{
    return da < db || (da == db && ia < ib);
}

/* ------------------------------------------------------------------------ */
/* Published counter-based generators. */
static uint64_t fnv1a64(const unsigned char *p, size_t n)
{
    uint64_t h = 0xcbf29ce484222325ULL;            /* FNV-64 offset basis */
    for (size_t i = 0; i < n; ++i) { h ^= p[i]; h *= 0x100000001b3ULL; } /* FNV-64 prime */
    return h;
}
static uint64_t splitmix64_out(uint64_t state, uint64_t j)
{
    uint64_t z = state + (j + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* ------------------------------------------------------------------------ */
orc_index *orc_create(int dim, int R, int metric, uint64_t seed)
{
    if (dim <= 0 || R <= 0 || (metric != ORC_L2 && metric != ORC_IP)) return NULL;
    orc_index *ix = calloc(1, sizeof *ix);
    if (!ix) return NULL;
    ix->dim = dim; ix->R = R; ix->metric = metric; ix->seed = seed;
    ix->beam_insert = 2 * R;
    ix->entry_samples = 0;
    ix->search_width = 1;
    ix->max_iters = 0;
    ix->repair_c = 8;
    ix->localized_repair = 1;
    ix->prune_cap = 0;   /* 0: no cap */
    ix->precision = ORC_P_FP32;
    ix->consolidate_frac = 0.2;
    ix->insert_batch_max = 10000;
    return ix;
}

void orc_destroy(orc_index *ix)
{
    if (!ix) return;
    free(ix->vec); free(ix->vec_lp); free(ix->vec_f32); free(ix->rows); free(ix->edge_d);
    free(ix->alive); free(ix->bg_changed); free(ix->bg_rows); free(ix->bg_rows_d);
    free(ix->log_rows); free(ix->log_d); free(ix);
}

/* Sec. 5.1 re-prunes a vertex's whole candidate list (its alive neighbours
 * plus what the update offers it) and bounds no list length, so by default
 * no candidate is cut.  A positive prune_cap keeps only that many nearest
 * candidates (an option for experiments, not the method). */
static int effective_prune_cap(const orc_index *ix)
{
    return ix->prune_cap > 0 ? ix->prune_cap : INT_MAX;
}

int orc_set(orc_index *ix, const char *key, double v)
{
    if (!strcmp(key, "beam_insert")) { if (v < ix->R || v > 512) return ORC_E_INVAL; ix->beam_insert = (int)v; }
    else if (!strcmp(key, "entry_samples")) { if (v < 0 || v > 4096) return ORC_E_INVAL; ix->entry_samples = (int)v; }
    else if (!strcmp(key, "search_width")) { if (v < 1 || v > 8) return ORC_E_INVAL; ix->search_width = (int)v; }
    else if (!strcmp(key, "max_iters")) { if (v < 0) return ORC_E_INVAL; ix->max_iters = (int)v; }
    else if (!strcmp(key, "repair_c")) { if (v < 1) return ORC_E_INVAL; ix->repair_c = (int)v; }
    else if (!strcmp(key, "prune_cap")) { if (v < 0) return ORC_E_INVAL; ix->prune_cap = (int)v; }
    else if (!strcmp(key, "consolidate_frac")) { if (v < 0 || v > 1) return ORC_E_INVAL; ix->consolidate_frac = v; }
    else if (!strcmp(key, "localized_repair")) { if (v != 0 && v != 1) return ORC_E_INVAL; ix->localized_repair = (int)v; }
    else if (!strcmp(key, "consolidate_async")) { if (v != 0 && v != 1) return ORC_E_INVAL; ix->consolidate_async = (int)v; }
    else if (!strcmp(key, "seed")) { ix->seed = (uint64_t)v; }
    else if (!strcmp(key, "insert_batch_max")) { if (v < 1) return ORC_E_INVAL; ix->insert_batch_max = (int64_t)v; }
    else if (!strcmp(key, "precision")) {
        if (v != 0 && v != 1 && v != 2 && v != 3) return ORC_E_INVAL;
        ix->precision = (int)v;
        for (int64_t i = 0; i < ix->n_slots; ++i)
            lp_vector(ix->precision, ix->vec_f32 + i * ix->dim, ix->dim, 0, ix->vec_lp + i * ix->dim);
    }
    else return ORC_E_INVAL;
    return ORC_OK;
}

int64_t orc_n_slots(const orc_index *ix) { return ix->n_slots; }
int64_t orc_n_alive(const orc_index *ix) { return ix->n_alive; }

static int reserve(orc_index *ix, int64_t need)
{
    if (need <= ix->cap) return ORC_OK;
    int64_t cap = ix->cap ? ix->cap : 1024;
    while (cap < need) cap *= 2;
    size_t d = (size_t)ix->dim, R = (size_t)ix->R;
    double *v = realloc(ix->vec, cap * d * sizeof(double));
    if (!v) return ORC_E_NOMEM;
    ix->vec = v;
    double *vl = realloc(ix->vec_lp, cap * d * sizeof(double));
    if (!vl) return ORC_E_NOMEM;
    ix->vec_lp = vl;
    float *vf = realloc(ix->vec_f32, cap * d * sizeof(float));
    if (!vf) return ORC_E_NOMEM;
    ix->vec_f32 = vf;
    int32_t *r = realloc(ix->rows, cap * R * sizeof(int32_t));
    if (!r) return ORC_E_NOMEM;
    ix->rows = r;
    double *e = realloc(ix->edge_d, cap * R * sizeof(double));
    if (!e) return ORC_E_NOMEM;
    ix->edge_d = e;
    uint8_t *a = realloc(ix->alive, cap);
    if (!a) return ORC_E_NOMEM;
    ix->alive = a;
    ix->cap = cap;
    return ORC_OK;
}

static void store_vectors(orc_index *ix, int64_t at, const float *v, int64_t n)
{
    int d = ix->dim;
    for (int64_t i = 0; i < n; ++i) {
        for (int j = 0; j < d; ++j) {
            float x = v[i * d + j];
            ix->vec_f32[(at + i) * d + j] = x;
            ix->vec[(at + i) * d + j] = (double)x;
        }
        lp_vector(ix->precision, v + i * d, d, 0, ix->vec_lp + (at + i) * d);
        for (int r = 0; r < ix->R; ++r) {
            ix->rows[(at + i) * ix->R + r] = ORC_INVALID;
            ix->edge_d[(at + i) * ix->R + r] = INFINITY;
        }
        ix->alive[at + i] = 0;
    }
}

/* ------------------------------------------------------------------------ */
/* Search -- Algorithm 1 (Sec. 4.2) on a single memory tier.
 *
 * Readings of what the algorithm leaves open:
 *  - InitCandidatePool: "random initialization".  Entry ids come from a
 *    SplitMix64 stream keyed by seed XOR FNV-1a(query bytes), so a query's
 *    entries never depend on its position in a batch.  Attempt j gives
 *    id = ((h_j >> 32) * n_slots) >> 32; ids that are deleted or were already
 *    drawn are skipped; drawing stops at min(E, n_alive) distinct ids or after
 *    8E + 64 attempts.  The best L of them by (d,id) start the pool.
 *  - GetNearest: the p (default 1) smallest unexpanded pool entries.
 *  - Update: pool <- the L smallest keys of pool U new; ids never repeat.
 *  - "until the pool is unchanged": stop once every pool entry has been
 *    expanded (or after max_iters iterations when that cap is set).
 *  - Deleted vertices are skipped: never entries, never evaluated, never
 *    expanded, never returned.  INVALID (-1) row slots are skipped.
 *  - Visited bookkeeping is exact here (one flag per id slot).
 */
typedef struct {
    double d; int32_t id; uint8_t expanded;
} pentry;

typedef struct {
    uint8_t *visited;     /* n_slots flags, cleared after each query */
    int32_t *touched; int64_t n_touched, cap_touched;
    pentry *pool, *merged, *fresh;
    int cap_pool;
} scratch_t;

static int scratch_init(scratch_t *s, int64_t n_slots, int L, int width, int R)
{
    memset(s, 0, sizeof *s);
    s->visited = calloc((size_t)(n_slots > 0 ? n_slots : 1), 1);
    s->cap_touched = 4096;
    s->touched = malloc(s->cap_touched * sizeof(int32_t));
    int cap = L + width * R + 8;
    int ecap = 8 * 4096 + 64;
    if (cap < ecap) cap = ecap;
    s->cap_pool = cap;
    s->pool = malloc(cap * sizeof(pentry));
    s->merged = malloc(cap * sizeof(pentry));
    s->fresh = malloc(cap * sizeof(pentry));
    return (s->visited && s->touched && s->pool && s->merged && s->fresh) ? 0 : -1;
}
static void scratch_free(scratch_t *s)
{
    free(s->visited); free(s->touched); free(s->pool); free(s->merged); free(s->fresh);
}
static void visit(scratch_t *s, int32_t id)
{
    s->visited[id] = 1;
    if (s->n_touched == s->cap_touched) {
        s->cap_touched *= 2;
        s->touched = realloc(s->touched, s->cap_touched * sizeof(int32_t));
    }
    s->touched[s->n_touched++] = id;
}
static void unvisit_all(scratch_t *s)
{
    for (int64_t i = 0; i < s->n_touched; ++i) s->visited[s->touched[i]] = 0;
    s->n_touched = 0;
}

static int cmp_pentry(const void *a, const void *b)
{
    const pentry *x = a, *y = b;
    if (key_less(x->d, x->id, y->d, y->id)) return -1;
    if (key_less(y->d, y->id, x->d, x->id)) return 1;
    return 0;
}

/* Relative gap between two keys, for the decisiveness margin. */
static double rel_gap(const orc_index *ix, double a, double b, double ip_scale)
{
    double g = fabs(a - b);
    double s = ix->metric == ORC_L2 ? fmax(fabs(a), fabs(b)) : ip_scale;
    return s > 0 ? g / s : g;
}

typedef struct {
    int64_t n_dist, n_exp, iters;
    double margin;   /* smallest relative gap among the comparisons that decided
                        the trajectory: entry cut, pool cut, parent choice */
} qstats;

/* One query.  q_exact/q_lp are the query in exact values and on the search
 * grid; qf are its FP32 words (for the entry hash).  n_slots and the alive
 * flags describe the snapshot searched.  Returns the final pool size, pool in
 * s->pool sorted by (d,id). */
static int search_one_t(const orc_index *ix, int64_t n_slots, const float *qf, const double *q_lp,
                        int L, int E, int width, int max_iters, scratch_t *s, qstats *st,
                        double ip_scale, int ktrack, int32_t *last_change);
static int search_one(const orc_index *ix, int64_t n_slots, const float *qf, const double *q_lp,
                      int L, int E, int width, int max_iters, scratch_t *s, qstats *st,
                      double ip_scale)
{
    return search_one_t(ix, n_slots, qf, q_lp, L, E, width, max_iters, s, st, ip_scale, 0, NULL);
}

/* ktrack > 0: *last_change receives the number of expansions done when the
 * ids of the first ktrack pool entries last changed (0: never after the
 * initial pool) -- the stopping step a predictor learns. */
static int search_one_t(const orc_index *ix, int64_t n_slots, const float *qf, const double *q_lp,
                        int L, int E, int width, int max_iters, scratch_t *s, qstats *st,
                        double ip_scale, int ktrack, int32_t *last_change)
{
    int32_t topk_before[64];
    int32_t lc = 0;
    const int d = ix->dim, R = ix->R;
    const double *V = ix->vec_lp;
    memset(st, 0, sizeof *st);
    st->margin = INFINITY;
    if (E <= 0) E = L;

    int64_t alive_in_snapshot = 0;
    for (int64_t i = 0; i < n_slots; ++i) alive_in_snapshot += ix->alive[i];

    /* InitCandidatePool: random entries from a per-query stream. */
    uint64_t key = ix->seed ^ fnv1a64((const unsigned char *)qf, (size_t)d * sizeof(float));
    int64_t want = E < alive_in_snapshot ? E : alive_in_snapshot;
    int64_t attempts = 8LL * E + 64;
    int ne = 0;
    for (int64_t j = 0; j < attempts && ne < want; ++j) {
        uint64_t h = splitmix64_out(key, (uint64_t)j);
        int64_t id = (int64_t)(((h >> 32) * (uint64_t)n_slots) >> 32);
        if (!ix->alive[id] || s->visited[id]) continue;
        visit(s, (int32_t)id);
        s->fresh[ne].id = (int32_t)id;
        s->fresh[ne].d = dist(ix->metric, q_lp, V + id * d, d);
        s->fresh[ne].expanded = 0;
        ++ne; ++st->n_dist;
    }
    qsort(s->fresh, ne, sizeof(pentry), cmp_pentry);
    if (ne > L) st->margin = fmin(st->margin, rel_gap(ix, s->fresh[L - 1].d, s->fresh[L].d, ip_scale));
    int np = ne < L ? ne : L;
    memcpy(s->pool, s->fresh, np * sizeof(pentry));

    /* Repeat: nearest unexpanded -> neighbours -> distances -> update. */
    for (;;) {
        if (max_iters > 0 && st->iters >= max_iters) break;
        int parents[8], npar = 0;
        for (int i = 0; i < np && npar < width; ++i)
            if (!s->pool[i].expanded) parents[npar++] = i;
        if (npar == 0) break;
        /* the next unexpanded entry after the chosen ones */
        for (int i = parents[npar - 1] + 1; i < np; ++i)
            if (!s->pool[i].expanded) {
                st->margin = fmin(st->margin, rel_gap(ix, s->pool[parents[npar - 1]].d, s->pool[i].d, ip_scale));
                break;
            }
        int nf = 0;
        for (int t = 0; t < npar; ++t) {
            pentry *pe = &s->pool[parents[t]];
            pe->expanded = 1;
            ++st->n_exp;
            const int32_t *row = ix->rows + (int64_t)pe->id * R;
            for (int r = 0; r < R; ++r) {
                int32_t u = row[r];
                if (u < 0 || u >= n_slots) continue;       /* INVALID slot */
                if (!ix->alive[u] || s->visited[u]) continue;
                visit(s, u);
                s->fresh[nf].id = u;
                s->fresh[nf].d = dist(ix->metric, q_lp, V + (int64_t)u * d, d);
                s->fresh[nf].expanded = 0;
                ++nf; ++st->n_dist;
            }
        }
        ++st->iters;
        int kt = ktrack < np ? ktrack : np;
        if (kt > 64) kt = 64;
        for (int t = 0; t < kt; ++t) topk_before[t] = s->pool[t].id;
        /* Update: merge and keep the L smallest keys. */
        memcpy(s->merged, s->pool, np * sizeof(pentry));
        memcpy(s->merged + np, s->fresh, nf * sizeof(pentry));
        int nm = np + nf;
        qsort(s->merged, nm, sizeof(pentry), cmp_pentry);
        if (nm > L) st->margin = fmin(st->margin, rel_gap(ix, s->merged[L - 1].d, s->merged[L].d, ip_scale));
        int np_new = nm < L ? nm : L;
        memcpy(s->pool, s->merged, np_new * sizeof(pentry));
        if (ktrack > 0) {
            int kn = ktrack < np_new ? ktrack : np_new;
            if (kn > 64) kn = 64;
            int changed = kn != kt;
            for (int t = 0; t < kn && !changed; ++t) changed = topk_before[t] != s->pool[t].id;
            if (changed) lc = (int32_t)st->iters;
        }
        np = np_new;
    }
    unvisit_all(s);
    if (last_change) *last_change = lc;
    return np;
}

static double max_norm(const orc_index *ix)
{
    double m = 0.0;
    for (int64_t i = 0; i < ix->n_slots; ++i) {
        if (!ix->alive[i]) continue;
        double s = 0.0;
        for (int j = 0; j < ix->dim; ++j) s += ix->vec[i * ix->dim + j] * ix->vec[i * ix->dim + j];
        if (s > m) m = s;
    }
    return sqrt(m);
}

/* Public batched search with optional threads (results never depend on the
 * thread count).  With rerank != 0 and a reduced search precision, the final
 * pool is re-scored with exact distances and re-sorted before taking k. */
typedef struct {
    const orc_index *ix; const float *q; int64_t lo, hi; int k, L, rerank;
    int32_t *ids; double *dd; int64_t *n_dist, *n_exp, *iters; double *margin; double xmax;
    int err;
} search_job;

static void *search_worker(void *arg)
{
    search_job *j = arg;
    const orc_index *ix = j->ix;
    const int d = ix->dim;
    scratch_t s;
    if (scratch_init(&s, ix->n_slots, j->L, ix->search_width, ix->R)) { j->err = ORC_E_NOMEM; return NULL; }
    double *q = malloc(sizeof(double) * d), *qlp = malloc(sizeof(double) * d);
    for (int64_t i = j->lo; i < j->hi; ++i) {
        const float *qf = j->q + i * d;
        double qn = 0.0;
        for (int t = 0; t < d; ++t) {
            q[t] = (double)qf[t]; qn += q[t] * q[t];
        }
        lp_vector(ix->precision, qf, d, 1, qlp);
        qstats st;
        int np = search_one(ix, ix->n_slots, qf, qlp, j->L, ix->entry_samples, ix->search_width,
                            ix->max_iters, &s, &st, sqrt(qn) * j->xmax);
        if (j->rerank && ix->precision != ORC_P_FP32) {
            for (int t = 0; t < np; ++t) s.pool[t].d = dist(ix->metric, q, ix->vec + (int64_t)s.pool[t].id * d, d);
            qsort(s.pool, np, sizeof(pentry), cmp_pentry);
        }
        for (int t = 0; t < j->k; ++t) {
            j->ids[i * j->k + t] = t < np ? s.pool[t].id : ORC_INVALID;
            j->dd[i * j->k + t] = t < np ? s.pool[t].d : INFINITY;
        }
        if (j->n_dist) j->n_dist[i] = st.n_dist;
        if (j->n_exp) j->n_exp[i] = st.n_exp;
        if (j->iters) j->iters[i] = st.iters;
        if (j->margin) j->margin[i] = st.margin;
    }
    free(q); free(qlp);
    scratch_free(&s);
    return NULL;
}

int orc_search(const orc_index *ix, const float *q, int64_t nq, int k, int L, int rerank,
               int32_t *ids, double *dd, int64_t *n_dist, int64_t *n_exp, int64_t *iters,
               double *margin, int nthreads)
{
    if (k < 1 || L < k || nq < 0) return ORC_E_INVAL;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > nq) nthreads = nq > 0 ? (int)nq : 1;
    double xmax = ix->metric == ORC_IP ? max_norm(ix) : 0.0;
    pthread_t th[256];
    search_job jobs[256];
    if (nthreads > 256) nthreads = 256;
    int64_t per = (nq + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = (search_job){ix, q, t * per, (t + 1) * per < nq ? (t + 1) * per : nq, k, L, rerank,
                               ids, dd, n_dist, n_exp, iters, margin, xmax, 0};
        if (jobs[t].lo > jobs[t].hi) jobs[t].lo = jobs[t].hi;
    }
    if (nthreads == 1) search_worker(&jobs[0]);
    else {
        for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, search_worker, &jobs[t]);
        for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    }
    for (int t = 0; t < nthreads; ++t) if (jobs[t].err) return jobs[t].err;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Exact kNN (Sec. 2.1 NNS definition; ground truth by exhaustive scan as in
 * the paper's evaluation): the k smallest (d,id) keys over the alive set. */
typedef struct {
    const float *base; int64_t n; int dim; const uint8_t *alive; int metric;
    const float *q; int64_t lo, hi; int k; int32_t *ids; double *dd;
} bf_job;

static void *bf_worker(void *arg)
{
    bf_job *j = arg;
    int d = j->dim;
    double *qd = malloc(sizeof(double) * d), *xd = malloc(sizeof(double) * d);
    pentry *best = malloc(sizeof(pentry) * (j->k + 1));
    for (int64_t i = j->lo; i < j->hi; ++i) {
        for (int t = 0; t < d; ++t) qd[t] = j->q[i * d + t];
        int nb = 0;
        for (int64_t u = 0; u < j->n; ++u) {
            if (j->alive && !j->alive[u]) continue;
            for (int t = 0; t < d; ++t) xd[t] = j->base[u * d + t];
            double du = dist(j->metric, qd, xd, d);
            if (nb == j->k && !key_less(du, (int32_t)u, best[nb - 1].d, best[nb - 1].id)) continue;
            int p = nb < j->k ? nb++ : nb - 1;   /* insertion into a sorted list */
            while (p > 0 && key_less(du, (int32_t)u, best[p - 1].d, best[p - 1].id)) { best[p] = best[p - 1]; --p; }
            best[p].d = du; best[p].id = (int32_t)u;
        }
        for (int t = 0; t < j->k; ++t) {
            j->ids[i * j->k + t] = t < nb ? best[t].id : ORC_INVALID;
            j->dd[i * j->k + t] = t < nb ? best[t].d : INFINITY;
        }
    }
    free(qd); free(xd); free(best);
    return NULL;
}

void orc_bruteforce(const float *base, int64_t n, int dim, const uint8_t *alive, int metric,
                    const float *q, int64_t nq, int k, int32_t *ids, double *dd, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (nq < nthreads) nthreads = nq > 0 ? (int)nq : 1;
    pthread_t th[256];
    bf_job jobs[256];
    int64_t per = (nq + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
        int64_t lo = t * per, hi = (t + 1) * per < nq ? (t + 1) * per : nq;
        if (lo > hi) lo = hi;
        jobs[t] = (bf_job){base, n, dim, alive, metric, q, lo, hi, k, ids, dd};
    }
    if (nthreads == 1) bf_worker(&jobs[0]);
    else {
        for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, bf_worker, &jobs[t]);
        for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    }
}

/* ------------------------------------------------------------------------ */
/* Rank-based candidate reordering (Sec. 5.1).
 * Input: m candidates c_0..c_{m-1} in (d,id) order.  For candidate i count
 * the earlier candidates j < i whose neighbour list contains c_i (a detour
 * c_j -> c_i exists); order the candidates by that count, ties by position
 * (a stable sort), and keep the first R.  The kept set is written in
 * candidate order, i.e. canonical (d,id) order, padded with INVALID/inf.
 * Reading: "previously selected neighbours" = all earlier candidates; a row
 * slot that is INVALID or deleted never matches (candidates are alive). */
typedef const int32_t *(*row_fn)(const void *ctx, int32_t id);

static int cmp_count_pos(const void *a, const void *b)
{
    const int64_t *x = a, *y = b;    /* (count << 32 | position) */
    return (*x > *y) - (*x < *y);
}

static void prune(int R, int m, const int32_t *cid, const double *cd, row_fn rows, const void *ctx,
                  int32_t *out_id, double *out_d)
{
    int64_t *ord = malloc(sizeof(int64_t) * (m > 0 ? m : 1));
    uint8_t *keep = calloc(m > 0 ? m : 1, 1);
    for (int i = 0; i < m; ++i) {
        int64_t cnt = 0;
        for (int j = 0; j < i; ++j) {
            const int32_t *row = rows(ctx, cid[j]);
            if (!row) continue;
            for (int r = 0; r < R; ++r) if (row[r] == cid[i]) { ++cnt; break; }
        }
        ord[i] = (cnt << 32) | i;
    }
    qsort(ord, m, sizeof(int64_t), cmp_count_pos);
    for (int t = 0; t < m && t < R; ++t) keep[ord[t] & 0xffffffff] = 1;
    int o = 0;
    for (int i = 0; i < m; ++i) if (keep[i]) { out_id[o] = cid[i]; out_d[o] = cd[i]; ++o; }
    for (; o < R; ++o) { out_id[o] = ORC_INVALID; out_d[o] = INFINITY; }
    free(ord); free(keep);
}

/* Snapshot of neighbour lists used while a batch is pruned. */
typedef struct {
    const int32_t *old_rows;   /* rows of ids < n_old */
    int64_t n_old;
    const int32_t *new_rows;   /* rows of ids in [n_old, n_old + n_new) */
    int64_t n_new;
    int R;
} snap_ctx;

static const int32_t *snap_row(const void *vctx, int32_t id)
{
    const snap_ctx *c = vctx;
    if (id < 0) return NULL;
    if (id < c->n_old) return c->old_rows + (int64_t)id * c->R;
    if (id < c->n_old + c->n_new && c->new_rows) return c->new_rows + (int64_t)(id - c->n_old) * c->R;
    return NULL;
}
static const int32_t *empty_row(const void *ctx, int32_t id) { (void)ctx; (void)id; return NULL; }

static int cmp_cand(const void *a, const void *b) { return cmp_pentry(a, b); }

/* ------------------------------------------------------------------------ */
/* Insertion of one batch (Sec. 5.1).
 * Readings: every vector of the batch searches the pre-batch graph with the
 * insertion pool size (batch-mates do not see each other); its candidate list
 * is that final pool; its forward row is the pruned list.  Reverse edges: for
 * every old vertex n named by some forward row, the candidates are n's alive
 * neighbours (stored distances) plus the new vertices pointing at it, all
 * of them in (d,id) order; they are pruned with the pre-batch
 * rows of old vertices and the forward rows of new ones.  All rows are
 * committed together at the end of the batch. */
typedef struct { int32_t v; double d; } incoming;
static void bg_log(orc_index *ix, const int32_t *fwd, const double *fwd_d, int64_t b);

static int insert_one_batch(orc_index *ix, const float *vecs, int64_t b, int32_t *out_ids)
{
    if (b < 0) return ORC_E_INVAL;
    if (b == 0) return ORC_OK;
    const int d = ix->dim, R = ix->R, Lins = ix->beam_insert;
    const int64_t n0 = ix->n_slots;
    int rc = reserve(ix, n0 + b);
    if (rc) return rc;
    store_vectors(ix, n0, vecs, b);

    int32_t *fwd = malloc(sizeof(int32_t) * b * R);
    double *fwd_d = malloc(sizeof(double) * b * R);
    scratch_t s;
    scratch_init(&s, n0 + b, Lins, ix->search_width, R);
    double xmax = ix->metric == ORC_IP ? max_norm(ix) : 0.0;
    int32_t *cid = malloc(sizeof(int32_t) * (Lins + 8));
    double *cdd = malloc(sizeof(double) * (Lins + 8));
    snap_ctx sc = {ix->rows, n0, NULL, 0, R};
    double *qlp = malloc(sizeof(double) * d);
    for (int64_t i = 0; i < b; ++i) {
        const int64_t v = n0 + i;
        qstats st;
        lp_vector(ix->precision, ix->vec_f32 + v * d, d, 1, qlp);
        int np = search_one(ix, n0, ix->vec_f32 + v * d, qlp, Lins, ix->entry_samples,
                            ix->search_width, 0, &s, &st, xmax);
        /* exact distances for the edges when the search ran on a coarser grid */
        if (ix->precision != ORC_P_FP32) {
            for (int t = 0; t < np; ++t) s.pool[t].d = dist(ix->metric, ix->vec + v * d, ix->vec + (int64_t)s.pool[t].id * d, d);
            qsort(s.pool, np, sizeof(pentry), cmp_pentry);
        }
        for (int t = 0; t < np; ++t) { cid[t] = s.pool[t].id; cdd[t] = s.pool[t].d; }
        prune(R, np, cid, cdd, snap_row, &sc, fwd + i * R, fwd_d + i * R);
    }
    free(cid); free(cdd); free(qlp);
    scratch_free(&s);

    /* Group reverse edges by target. */
    int64_t *cnt = calloc(n0 + 1, sizeof(int64_t));
    for (int64_t i = 0; i < b * R; ++i) if (fwd[i] >= 0) cnt[fwd[i]]++;
    int64_t *off = malloc(sizeof(int64_t) * (n0 + 1));
    off[0] = 0;
    for (int64_t t = 0; t < n0; ++t) off[t + 1] = off[t] + cnt[t];
    incoming *inc = malloc(sizeof(incoming) * (off[n0] + 1));
    int64_t *cur = malloc(sizeof(int64_t) * (n0 + 1));
    memcpy(cur, off, sizeof(int64_t) * (n0 + 1));
    for (int64_t i = 0; i < b; ++i)
        for (int r = 0; r < R; ++r) {
            int32_t t = fwd[i * R + r];
            if (t >= 0) inc[cur[t]++] = (incoming){(int32_t)(n0 + i), fwd_d[i * R + r]};
        }

    /* Reverse prune of every target against the same snapshot. */
    snap_ctx sc2 = {ix->rows, n0, fwd, b, R};
    int cap = effective_prune_cap(ix);
    int64_t n_targets = 0;
    for (int64_t t = 0; t < n0; ++t) if (cnt[t]) ++n_targets;
    int32_t *tgt = malloc(sizeof(int32_t) * (n_targets + 1));
    int32_t *trow = malloc(sizeof(int32_t) * (n_targets + 1) * R);
    double *trow_d = malloc(sizeof(double) * (n_targets + 1) * R);
    pentry *cl = malloc(sizeof(pentry) * (R + b + 1));
    int32_t *pid = malloc(sizeof(int32_t) * (R + b + 1));
    double *pdd = malloc(sizeof(double) * (R + b + 1));
    int64_t ti = 0;
    for (int64_t t = 0; t < n0; ++t) {
        if (!cnt[t]) continue;
        int m = 0;
        for (int r = 0; r < R; ++r) {
            int32_t u = ix->rows[t * R + r];
            if (u >= 0 && ix->alive[u]) { cl[m].id = u; cl[m].d = ix->edge_d[t * R + r]; ++m; }
        }
        for (int64_t e = off[t]; e < off[t + 1]; ++e) { cl[m].id = inc[e].v; cl[m].d = inc[e].d; ++m; }
        qsort(cl, m, sizeof(pentry), cmp_cand);
        if (m > cap) m = cap;
        for (int i = 0; i < m; ++i) { pid[i] = cl[i].id; pdd[i] = cl[i].d; }
        prune(R, m, pid, pdd, snap_row, &sc2, trow + ti * R, trow_d + ti * R);
        tgt[ti++] = (int32_t)t;
    }
    if (ix->bg_active) bg_log(ix, fwd, fwd_d, b);
    /* Commit. */
    for (int64_t i = 0; i < n_targets; ++i) {
        memcpy(ix->rows + (int64_t)tgt[i] * R, trow + i * R, sizeof(int32_t) * R);
        memcpy(ix->edge_d + (int64_t)tgt[i] * R, trow_d + i * R, sizeof(double) * R);
    }
    for (int64_t i = 0; i < b; ++i) {
        memcpy(ix->rows + (n0 + i) * R, fwd + i * R, sizeof(int32_t) * R);
        memcpy(ix->edge_d + (n0 + i) * R, fwd_d + i * R, sizeof(double) * R);
        ix->alive[n0 + i] = 1;
        if (out_ids) out_ids[i] = (int32_t)(n0 + i);
    }
    ix->n_slots = n0 + b;
    ix->n_alive += b;
    free(cnt); free(off); free(inc); free(cur); free(tgt); free(trow); free(trow_d);
    free(cl); free(pid); free(pdd); free(fwd); free(fwd_d);
    return ORC_OK;
}

int orc_build(orc_index *ix, const float *vecs, int64_t n, int64_t batch_max);

/* Insertion of n vectors: into an empty index this is the build rule below;
 * otherwise consecutive batches of at most insert_batch_max vectors. */
int orc_insert(orc_index *ix, const float *vecs, int64_t n, int32_t *out_ids)
{
    if (n < 0) return ORC_E_INVAL;
    if (n == 0) return ORC_OK;
    if (ix->n_slots == 0) {
        int rc = orc_build(ix, vecs, n, ix->insert_batch_max);
        if (!rc && out_ids) for (int64_t i = 0; i < n; ++i) out_ids[i] = (int32_t)i;
        return rc;
    }
    for (int64_t done = 0; done < n;) {
        int64_t b = n - done < ix->insert_batch_max ? n - done : ix->insert_batch_max;
        int rc = insert_one_batch(ix, vecs + done * ix->dim, b, out_ids ? out_ids + done : NULL);
        if (rc) return rc;
        done += b;
    }
    return ORC_OK;
}

/* Seed graph: the first S0 = min(n, 4R) vectors, each row pruned from all the
 * other seed vectors with empty neighbour lists, so every detour count is 0
 * and each row is the exact R-nearest list among the seed.  The remaining
 * vectors follow in batches of min(batch_max, ceil(n_alive / 8)). */
int orc_build(orc_index *ix, const float *vecs, int64_t n, int64_t batch_max)
{
    if (n <= 0 || ix->n_slots != 0 || batch_max < 1) return ORC_E_INVAL;
    const int d = ix->dim, R = ix->R;
    int64_t s0 = n < 4 * R ? n : 4 * R;
    int rc = reserve(ix, n);
    if (rc) return rc;
    store_vectors(ix, 0, vecs, s0);
    pentry *cl = malloc(sizeof(pentry) * s0);
    int32_t *pid = malloc(sizeof(int32_t) * s0);
    double *pdd = malloc(sizeof(double) * s0);
    for (int64_t v = 0; v < s0; ++v) {
        int m = 0;
        for (int64_t u = 0; u < s0; ++u) {
            if (u == v) continue;
            cl[m].id = (int32_t)u;
            cl[m].d = dist(ix->metric, ix->vec + v * d, ix->vec + u * d, d);
            ++m;
        }
        qsort(cl, m, sizeof(pentry), cmp_cand);
        for (int i = 0; i < m; ++i) { pid[i] = cl[i].id; pdd[i] = cl[i].d; }
        prune(R, m, pid, pdd, empty_row, NULL, ix->rows + v * R, ix->edge_d + v * R);
    }
    for (int64_t v = 0; v < s0; ++v) ix->alive[v] = 1;
    ix->n_slots = s0;
    ix->n_alive = s0;
    free(cl); free(pid); free(pdd);
    int64_t done = s0;
    while (done < n) {
        int64_t b = (ix->n_alive + 7) / 8;
        if (b > batch_max) b = batch_max;
        if (b > n - done) b = n - done;
        rc = insert_one_batch(ix, vecs + done * d, b, NULL);
        if (rc) return rc;
        done += b;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Deletion (Sec. 5.2): mark, then repair.
 * Readings: V^L holds alive vertices whose valid neighbour slots are more
 * than half deleted.  For v in V^L the candidates are its alive neighbours
 * (stored distances) and, for each deleted neighbour p in row order, the
 * first c entries of p's row that are alive, not v and not yet candidates.
 * If fewer than R candidates result, the pool of a search for v's own vector
 * (insertion pool size, same snapshot) tops them up.  All candidates are put
 * in (d,id) order and pruned with the pre-repair rows.
 * Consolidation uses the same routine with "at least one deleted neighbour"
 * and c = R.  It runs when the deleted fraction since the last consolidation
 * reaches consolidate_frac (the paper's example threshold is 20%). */
static void repair_compute(orc_index *ix, int consolidate, int32_t *out, double *out_d, uint8_t *changed)
{
    const int d = ix->dim, R = ix->R;
    const int64_t n = ix->n_slots;
    const int c = consolidate ? R : ix->repair_c;
    int32_t *pre = malloc(sizeof(int32_t) * n * R);
    memcpy(pre, ix->rows, sizeof(int32_t) * n * R);
    snap_ctx sc = {pre, n, NULL, 0, R};
    int cap = effective_prune_cap(ix);
    int maxc = R + R * c + ix->beam_insert + 1;
    pentry *cl = malloc(sizeof(pentry) * maxc);
    int32_t *pid = malloc(sizeof(int32_t) * maxc);
    double *pdd = malloc(sizeof(double) * maxc);
    uint8_t *incand = calloc(n, 1);
    scratch_t s;
    scratch_init(&s, n, ix->beam_insert, ix->search_width, R);
    double xmax = ix->metric == ORC_IP ? max_norm(ix) : 0.0;
    for (int64_t v = 0; v < n; ++v) {
        if (!ix->alive[v]) continue;
        int valid = 0, del = 0;
        for (int r = 0; r < R; ++r) {
            int32_t u = pre[v * R + r];
            if (u < 0) continue;
            ++valid;
            if (!ix->alive[u]) ++del;
        }
        int affected = consolidate ? del >= 1 : 2 * del > valid;
        if (!affected) continue;
        int m = 0;
        for (int r = 0; r < R; ++r) {
            int32_t u = pre[v * R + r];
            if (u >= 0 && ix->alive[u]) { cl[m].id = u; cl[m].d = ix->edge_d[v * R + r]; incand[u] = 1; ++m; }
        }
        for (int r = 0; r < R; ++r) {
            int32_t p = pre[v * R + r];
            if (p < 0 || ix->alive[p]) continue;
            int taken = 0;
            for (int e = 0; e < R && taken < c; ++e) {
                int32_t u = pre[(int64_t)p * R + e];
                if (u < 0 || !ix->alive[u] || u == v || incand[u]) continue;
                cl[m].id = u;
                cl[m].d = dist(ix->metric, ix->vec + v * d, ix->vec + (int64_t)u * d, d);
                incand[u] = 1; ++m; ++taken;
            }
        }
        if (m < R) {
            qstats st;
            double *qlp = malloc(sizeof(double) * d);
            lp_vector(ix->precision, ix->vec_f32 + v * d, d, 1, qlp);
            int np = search_one(ix, n, ix->vec_f32 + v * d, qlp, ix->beam_insert,
                                ix->entry_samples, ix->search_width, 0, &s, &st, xmax);
            for (int t = 0; t < np; ++t) {
                int32_t u = s.pool[t].id;
                if (u == v || incand[u]) continue;
                cl[m].id = u;
                cl[m].d = dist(ix->metric, ix->vec + v * d, ix->vec + (int64_t)u * d, d);
                incand[u] = 1; ++m;
            }
            free(qlp);
        }
        for (int i = 0; i < m; ++i) incand[cl[i].id] = 0;
        qsort(cl, m, sizeof(pentry), cmp_cand);
        if (m > cap) m = cap;
        for (int i = 0; i < m; ++i) { pid[i] = cl[i].id; pdd[i] = cl[i].d; }
        prune(R, m, pid, pdd, snap_row, &sc, out + v * R, out_d + v * R);
        changed[v] = 1;
    }
    scratch_free(&s);
    free(pre); free(cl); free(pid); free(pdd); free(incand);
}

static void commit_rows(orc_index *ix, int64_t n, const int32_t *out, const double *out_d,
                        const uint8_t *changed)
{
    const int R = ix->R;
    for (int64_t v = 0; v < n; ++v) if (changed[v]) {
        memcpy(ix->rows + v * R, out + v * R, sizeof(int32_t) * R);
        memcpy(ix->edge_d + v * R, out_d + v * R, sizeof(double) * R);
    }
}

static void repair(orc_index *ix, int consolidate)
{
    const int64_t n = ix->n_slots, R = ix->R;
    int32_t *out = malloc(sizeof(int32_t) * n * R);
    double *out_d = malloc(sizeof(double) * n * R);
    uint8_t *changed = calloc(n, 1);
    repair_compute(ix, consolidate, out, out_d, changed);
    commit_rows(ix, n, out, out_d, changed);
    free(out); free(out_d); free(changed);
}

/* Consolidation in the background (Sec. 5.3), written out sequentially: a
 * consolidation on a snapshot equals one computed when the snapshot is
 * taken, so bg_begin computes it then and keeps the rows staged.  Insertion
 * batches meanwhile append their forward rows to a log (their ids follow the
 * snapshot's in order).  The merge writes the staged rows, then re-prunes
 * every rewritten row that the logged rows name, with the candidates a
 * reverse-edge update uses (its alive entries with their stored distances,
 * then the logged vertices pointing at it, all in (d,id) order), against
 * the rows as they stand after the first step; all re-pruned
 * rows are written at the end.  Other rows keep their live state. */
static void bg_begin(orc_index *ix)
{
    const int64_t n = ix->n_slots, R = ix->R;
    ix->bg_n0 = n;
    ix->bg_rows = malloc(sizeof(int32_t) * (n * R + 1));
    ix->bg_rows_d = malloc(sizeof(double) * (n * R + 1));
    ix->bg_changed = calloc(n + 1, 1);
    repair_compute(ix, 1, ix->bg_rows, ix->bg_rows_d, ix->bg_changed);
    ix->log_n = 0;
    ix->bg_active = 1;
}

static void bg_log(orc_index *ix, const int32_t *fwd, const double *fwd_d, int64_t b)
{
    const int R = ix->R;
    if (ix->log_n + b > ix->log_cap) {
        int64_t cap = ix->log_n + b > 2 * ix->log_cap ? ix->log_n + b : 2 * ix->log_cap;
        ix->log_rows = realloc(ix->log_rows, sizeof(int32_t) * cap * R);
        ix->log_d = realloc(ix->log_d, sizeof(double) * cap * R);
        ix->log_cap = cap;
    }
    memcpy(ix->log_rows + ix->log_n * R, fwd, sizeof(int32_t) * b * R);
    memcpy(ix->log_d + ix->log_n * R, fwd_d, sizeof(double) * b * R);
    ix->log_n += b;
}

int orc_consolidate_wait(orc_index *ix)
{
    if (!ix->bg_active) return ORC_OK;
    ix->bg_active = 0;
    const int R = ix->R;
    const int64_t n0 = ix->bg_n0, n = ix->n_slots;
    commit_rows(ix, n0, ix->bg_rows, ix->bg_rows_d, ix->bg_changed);
    if (ix->log_n > 0) {
        int64_t *cnt = calloc(n0 + 1, sizeof(int64_t));
        for (int64_t i = 0; i < ix->log_n * R; ++i) {
            int32_t t = ix->log_rows[i];
            if (t >= 0 && t < n0 && ix->bg_changed[t]) cnt[t]++;
        }
        int64_t *off = malloc(sizeof(int64_t) * (n0 + 1));
        off[0] = 0;
        for (int64_t t = 0; t < n0; ++t) off[t + 1] = off[t] + cnt[t];
        incoming *inc = malloc(sizeof(incoming) * (off[n0] + 1));
        int64_t *cur = malloc(sizeof(int64_t) * (n0 + 1));
        memcpy(cur, off, sizeof(int64_t) * (n0 + 1));
        for (int64_t i = 0; i < ix->log_n; ++i)
            for (int r = 0; r < R; ++r) {
                int32_t t = ix->log_rows[i * R + r];
                if (t >= 0 && t < n0 && ix->bg_changed[t])
                    inc[cur[t]++] = (incoming){(int32_t)(n0 + i), ix->log_d[i * R + r]};
            }
        int32_t *pre = malloc(sizeof(int32_t) * n * R);
        memcpy(pre, ix->rows, sizeof(int32_t) * n * R);
        snap_ctx sc = {pre, n, NULL, 0, R};
        int cap = effective_prune_cap(ix);
        int64_t maxin = 0;
        for (int64_t t = 0; t < n0; ++t) if (cnt[t] > maxin) maxin = cnt[t];
        pentry *cl = malloc(sizeof(pentry) * (R + maxin + 1));
        int32_t *pid = malloc(sizeof(int32_t) * (R + maxin + 1));
        double *pdd = malloc(sizeof(double) * (R + maxin + 1));
        int32_t *trow = malloc(sizeof(int32_t) * n0 * R + 1);
        double *trow_d = malloc(sizeof(double) * n0 * R + 1);
        uint8_t *hit = calloc(n0 + 1, 1);
        for (int64_t t = 0; t < n0; ++t) {
            if (!cnt[t]) continue;
            int m = 0;
            for (int r = 0; r < R; ++r) {
                int32_t u = pre[t * R + r];
                if (u >= 0 && ix->alive[u]) { cl[m].id = u; cl[m].d = ix->edge_d[t * R + r]; ++m; }
            }
            for (int64_t e = off[t]; e < off[t + 1]; ++e) { cl[m].id = inc[e].v; cl[m].d = inc[e].d; ++m; }
            qsort(cl, m, sizeof(pentry), cmp_cand);
            if (m > cap) m = cap;
            for (int i = 0; i < m; ++i) { pid[i] = cl[i].id; pdd[i] = cl[i].d; }
            prune(R, m, pid, pdd, snap_row, &sc, trow + t * R, trow_d + t * R);
            hit[t] = 1;
        }
        commit_rows(ix, n0, trow, trow_d, hit);
        free(cnt); free(off); free(inc); free(cur); free(pre); free(cl); free(pid); free(pdd);
        free(trow); free(trow_d); free(hit);
    }
    free(ix->bg_rows); free(ix->bg_rows_d); free(ix->bg_changed);
    ix->bg_rows = NULL; ix->bg_rows_d = NULL; ix->bg_changed = NULL;
    ix->log_n = 0;
    return ORC_OK;
}

int orc_delete(orc_index *ix, const int32_t *ids, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) if (ids[i] < 0 || ids[i] >= ix->n_slots) return ORC_E_NOTFOUND;
    int64_t newly = 0;
    for (int64_t i = 0; i < n; ++i) if (ix->alive[ids[i]]) { ix->alive[ids[i]] = 0; ++newly; }
    if (ix->alive_at_consolidate == 0) ix->alive_at_consolidate = ix->n_alive;
    ix->n_alive -= newly;
    ix->deleted_since += newly;
    if (newly == 0) return ORC_OK;
    /* The paper's deletion ablation separates the three parts: lazy deletion
     * alone (no repair, consolidate_frac 0 = never), lazy deletion with global
     * consolidation, and both with localized repair (the method). */
    int due = ix->consolidate_frac > 0 &&
              (double)ix->deleted_since >= ix->consolidate_frac * (double)ix->alive_at_consolidate;
    if (due && ix->consolidate_async && !ix->bg_active) {
        bg_begin(ix);
        ix->deleted_since = 0;
        ix->alive_at_consolidate = ix->n_alive;
    } else if (due && !ix->consolidate_async) {
        orc_consolidate_wait(ix);
        repair(ix, 1);
        ix->deleted_since = 0;
        ix->alive_at_consolidate = ix->n_alive;
    } else if (ix->localized_repair) {
        repair(ix, 0);   /* a due consolidation waits for the pending one */
    }
    return ORC_OK;
}

int orc_consolidate(orc_index *ix)
{
    orc_consolidate_wait(ix);
    repair(ix, 1);
    ix->deleted_since = 0;
    ix->alive_at_consolidate = ix->n_alive;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* State transfer (for starting another implementation from this state). */
int orc_export(const orc_index *ix, int32_t *rows, double *edge_d, uint8_t *alive)
{
    int64_t n = ix->n_slots;
    if (rows) memcpy(rows, ix->rows, sizeof(int32_t) * n * ix->R);
    if (edge_d) memcpy(edge_d, ix->edge_d, sizeof(double) * n * ix->R);
    if (alive) memcpy(alive, ix->alive, n);
    return ORC_OK;
}

int orc_import(orc_index *ix, const float *vecs, int64_t n, const int32_t *rows,
               const double *edge_d, const uint8_t *alive)
{
    if (ix->n_slots != 0 || n < 0) return ORC_E_INVAL;
    int rc = reserve(ix, n > 0 ? n : 1);
    if (rc) return rc;
    store_vectors(ix, 0, vecs, n);
    memcpy(ix->rows, rows, sizeof(int32_t) * n * ix->R);
    memcpy(ix->edge_d, edge_d, sizeof(double) * n * ix->R);
    int64_t na = 0;
    for (int64_t i = 0; i < n; ++i) { ix->alive[i] = alive[i] ? 1 : 0; na += ix->alive[i]; }
    ix->n_slots = n;
    ix->n_alive = na;
    return ORC_OK;
}

/* Exact distance between two stored vectors (for checks of edge distances). */
double orc_dist_ids(const orc_index *ix, int32_t a, int32_t b)
{
    return dist(ix->metric, ix->vec + (int64_t)a * ix->dim, ix->vec + (int64_t)b * ix->dim, ix->dim);
}

/* The value grids, exposed so tests can pin them against published formats. */
double orc_round_fp16(double x) { return to_fp16(x); }
double orc_round_bf16(double x) { return to_bf16(x); }
double orc_round_e4m3(double x) { return to_e4m3(x); }
/* The FP8 form of n vectors: per-vector scale and the reconstructed values
 * (stored-vector form, or query form when is_query != 0). */
void orc_fp8_vectors(const float *x, int64_t n, int d, int is_query, float *scale, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        scale[i] = fp8_scale(x + i * d, d);
        lp_vector(ORC_P_FP8, x + i * d, d, is_query, out + i * d);
    }
}
uint64_t orc_fnv1a64(const unsigned char *p, int64_t n) { return fnv1a64(p, (size_t)n); }
uint64_t orc_splitmix64(uint64_t state, uint64_t j) { return splitmix64_out(state, j); }

/* Rank-based reordering on an explicit candidate list and an explicit table
 * of neighbour lists (n_rows x R, INVALID = -1), for hand-worked checks. */
typedef struct { const int32_t *tab; int64_t n; int R; } table_ctx;
static const int32_t *table_row(const void *vctx, int32_t id)
{
    const table_ctx *c = vctx;
    if (id < 0 || id >= c->n) return NULL;
    return c->tab + (int64_t)id * c->R;
}
void orc_prune_explicit(int R, int m, const int32_t *cid, const double *cd, const int32_t *tab,
                        int64_t n_rows, int32_t *out_id, double *out_d)
{
    table_ctx c = {tab, n_rows, R};
    prune(R, m, cid, cd, table_row, &c, out_id, out_d);
}

/* Exact distances of queries to given ids (nq x k; id -1 gives +inf). */
void orc_query_dists(const orc_index *ix, const float *q, int64_t nq, int k, const int32_t *ids, double *out)
{
    int d = ix->dim;
    double *qd = malloc(sizeof(double) * d);
    for (int64_t i = 0; i < nq; ++i) {
        for (int t = 0; t < d; ++t) qd[t] = q[i * d + t];
        for (int j = 0; j < k; ++j) {
            int32_t u = ids[i * k + j];
            out[i * k + j] = (u < 0 || u >= ix->n_slots) ? INFINITY
                             : dist(ix->metric, qd, ix->vec + (int64_t)u * d, d);
        }
    }
    free(qd);
}

/* ------------------------------------------------------------------------ */
/* Search with caller-given entry points and per-query expansion caps.
 * entries: nq x ecap ids (-1 = none); every distinct alive id of a query's
 * list is evaluated and the best L of them by (d,id) start its pool (a list
 * with no usable id leaves the random initialisation).  max_iters: nq caps (0 = none).  The
 * rest is the search above.  This is how predicted entry points and a
 * predicted stopping step enter the method (random entry points being one
 * choice among algorithm-supplied ones, Sec. 2.3). */
static int search_one_listed(const orc_index *ix, const float *qf, const double *q_lp, int L,
                             const int32_t *list, int ecap, int max_iters, scratch_t *s,
                             qstats *st, int32_t *last_change)
{
    const int d = ix->dim, R = ix->R;
    const double *V = ix->vec_lp;
    memset(st, 0, sizeof *st);
    st->margin = INFINITY;
    int ne = 0;
    for (int j = 0; j < ecap; ++j) {
        int32_t id = list[j];
        if (id < 0 || id >= ix->n_slots || !ix->alive[id] || s->visited[id]) continue;
        visit(s, id);
        s->fresh[ne].id = id;
        s->fresh[ne].d = dist(ix->metric, q_lp, V + (int64_t)id * d, d);
        s->fresh[ne].expanded = 0;
        ++ne; ++st->n_dist;
    }
    if (ne == 0) {
        unvisit_all(s);
        double xm = 0.0;
        int np = search_one(ix, ix->n_slots, qf, q_lp, L, ix->entry_samples, ix->search_width,
                            max_iters, s, st, xm);
        if (last_change) *last_change = -1;
        return np;
    }
    qsort(s->fresh, ne, sizeof(pentry), cmp_pentry);
    int np = ne < L ? ne : L;
    memcpy(s->pool, s->fresh, np * sizeof(pentry));
    int32_t lc = 0;
    for (;;) {
        if (max_iters > 0 && st->iters >= max_iters) break;
        int parents[8], npar = 0;
        for (int i = 0; i < np && npar < ix->search_width; ++i)
            if (!s->pool[i].expanded) parents[npar++] = i;
        if (npar == 0) break;
        int nf = 0;
        for (int t = 0; t < npar; ++t) {
            s->pool[parents[t]].expanded = 1;
            ++st->n_exp;
            const int32_t *row = ix->rows + (int64_t)s->pool[parents[t]].id * R;
            for (int r = 0; r < R; ++r) {
                int32_t u = row[r];
                if (u < 0 || u >= ix->n_slots || !ix->alive[u] || s->visited[u]) continue;
                visit(s, u);
                s->fresh[nf].id = u;
                s->fresh[nf].d = dist(ix->metric, q_lp, V + (int64_t)u * d, d);
                s->fresh[nf].expanded = 0;
                ++nf; ++st->n_dist;
            }
        }
        ++st->iters;
        memcpy(s->merged, s->pool, np * sizeof(pentry));
        memcpy(s->merged + np, s->fresh, nf * sizeof(pentry));
        int nm = np + nf;
        qsort(s->merged, nm, sizeof(pentry), cmp_pentry);
        np = nm < L ? nm : L;
        memcpy(s->pool, s->merged, np * sizeof(pentry));
    }
    unvisit_all(s);
    if (last_change) *last_change = lc;
    return np;
}

/* Plain search that also reports, per query, the expansion count after which
 * its top-k never changed (the stopping-step label of the predictor). */
int orc_search_trace(const orc_index *ix, const float *q, int64_t nq, int k, int L,
                     int32_t *ids, int32_t *last_change)
{
    if (k < 1 || L < k || k > 64) return ORC_E_INVAL;
    scratch_t s;
    if (scratch_init(&s, ix->n_slots, L, ix->search_width, ix->R)) return ORC_E_NOMEM;
    const int d = ix->dim;
    double *qlp = malloc(sizeof(double) * d);
    for (int64_t i = 0; i < nq; ++i) {
        const float *qf = q + i * d;
        lp_vector(ix->precision, qf, d, 1, qlp);
        qstats st;
        int np = search_one_t(ix, ix->n_slots, qf, qlp, L, ix->entry_samples, ix->search_width,
                              ix->max_iters, &s, &st, 0.0, k, last_change + i);
        for (int t = 0; t < k; ++t) ids[i * k + t] = t < np ? s.pool[t].id : ORC_INVALID;
    }
    free(qlp);
    scratch_free(&s);
    return ORC_OK;
}

int orc_search_listed(const orc_index *ix, const float *q, int64_t nq, int k, int L,
                      const int32_t *entries, int ecap, const int32_t *max_iters,
                      int32_t *ids, double *dd, int64_t *n_exp)
{
    if (k < 1 || L < k) return ORC_E_INVAL;
    scratch_t s;
    if (scratch_init(&s, ix->n_slots, L, ix->search_width, ix->R)) return ORC_E_NOMEM;
    const int d = ix->dim;
    double *qlp = malloc(sizeof(double) * d);
    for (int64_t i = 0; i < nq; ++i) {
        const float *qf = q + i * d;
        lp_vector(ix->precision, qf, d, 1, qlp);
        qstats st;
        int np = search_one_listed(ix, qf, qlp, L, entries + i * ecap, ecap,
                                   max_iters ? max_iters[i] : 0, &s, &st, NULL);
        for (int t = 0; t < k; ++t) {
            ids[i * k + t] = t < np ? s.pool[t].id : ORC_INVALID;
            dd[i * k + t] = t < np ? s.pool[t].d : INFINITY;
        }
        if (n_exp) n_exp[i] = st.n_exp;
    }
    free(qlp);
    scratch_free(&s);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The gating of the learned form (an extension of the method: entry points
 * supplied by a separate algorithm, Sec. 2.3, and a stop before Alg. 1 has
 * expanded everything).  From a query's outputs z (nc cluster logits, then
 * the predicted log stop step): the cluster is the first largest logit; its
 * softmax probability p = 1 / sum_j exp(z_j - z_max); with p >= conf the
 * query starts from that cluster's entry list and its expansions are capped
 * at max(min_iters, ceil(stop_scale * exp(min(z_nc, 20)))), the ceiling held
 * at or below 2^30; otherwise it runs plain search (cluster -1, no cap). */
void orc_model_decide(const double *z, int64_t n, int nc, double conf, double stop_scale,
                      int min_iters, int32_t *q_entry, int32_t *q_max)
{
    for (int64_t i = 0; i < n; ++i) {
        const double *zi = z + i * (nc + 1);
        int best = 0;
        for (int j = 1; j < nc; ++j)
            if (zi[j] > zi[best]) best = j;
        double se = 0.0;
        for (int j = 0; j < nc; ++j) se += exp(zi[j] - zi[best]);
        const double p = 1.0 / se;
        if (p >= conf) {
            double cap = ceil(stop_scale * exp(zi[nc] < 20.0 ? zi[nc] : 20.0));
            if (cap > 1073741824.0) cap = 1073741824.0;
            q_entry[i] = best;
            q_max[i] = cap < (double)min_iters ? min_iters : (int32_t)cap;
        } else {
            q_entry[i] = -1;
            q_max[i] = 0;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* The entry/stop predictor: a multilayer perceptron din -> h -> h -> nc + 1
 * with ReLU, FP64 here.  Outputs 0..nc-1 are logits of the entry cluster,
 * output nc predicts log(stop step).  Loss per sample: softmax cross-entropy
 * on the cluster label plus lambda * Huber(z_nc - log_stop; delta); the batch
 * loss is the mean.  Weights are row-major (in x out). */
typedef struct {
    int din, h, nc;
    const double *w1, *b1, *w2, *b2, *w3, *b3;
} mlp_view;

static void mlp_fwd_one(const mlp_view *m, const double *x, double *h1, double *h2, double *z)
{
    const int din = m->din, h = m->h, no = m->nc + 1;
    for (int j = 0; j < h; ++j) {
        double s = m->b1[j];
        for (int i = 0; i < din; ++i) s += x[i] * m->w1[i * h + j];
        h1[j] = s > 0 ? s : 0;
    }
    for (int j = 0; j < h; ++j) {
        double s = m->b2[j];
        for (int i = 0; i < h; ++i) s += h1[i] * m->w2[i * h + j];
        h2[j] = s > 0 ? s : 0;
    }
    for (int j = 0; j < no; ++j) {
        double s = m->b3[j];
        for (int i = 0; i < h; ++i) s += h2[i] * m->w3[i * no + j];
        z[j] = s;
    }
}

void orc_mlp_forward(int din, int h, int nc, const double *w1, const double *b1, const double *w2,
                     const double *b2, const double *w3, const double *b3, const double *x,
                     int64_t n, double *out)
{
    mlp_view m = {din, h, nc, w1, b1, w2, b2, w3, b3};
    double *h1 = malloc(sizeof(double) * h), *h2 = malloc(sizeof(double) * h);
    for (int64_t i = 0; i < n; ++i) mlp_fwd_one(&m, x + i * din, h1, h2, out + i * (nc + 1));
    free(h1); free(h2);
}

double orc_mlp_loss_grad(int din, int h, int nc, const double *w1, const double *b1,
                         const double *w2, const double *b2, const double *w3, const double *b3,
                         const double *x, const int32_t *label, const double *log_stop, int64_t n,
                         double lambda, double delta, double *g1, double *gb1, double *g2,
                         double *gb2, double *g3, double *gb3)
{
    mlp_view m = {din, h, nc, w1, b1, w2, b2, w3, b3};
    const int no = nc + 1;
    memset(g1, 0, sizeof(double) * din * h); memset(gb1, 0, sizeof(double) * h);
    memset(g2, 0, sizeof(double) * h * h);   memset(gb2, 0, sizeof(double) * h);
    memset(g3, 0, sizeof(double) * h * no);  memset(gb3, 0, sizeof(double) * no);
    double *h1 = malloc(sizeof(double) * h), *h2 = malloc(sizeof(double) * h);
    double *z = malloc(sizeof(double) * no), *dz = malloc(sizeof(double) * no);
    double *dh2 = malloc(sizeof(double) * h), *dh1 = malloc(sizeof(double) * h);
    double loss = 0.0;
    for (int64_t s = 0; s < n; ++s) {
        const double *xs = x + s * din;
        mlp_fwd_one(&m, xs, h1, h2, z);
        /* cross-entropy over the nc logits (shifted by the max for range) */
        double mx = z[0];
        for (int j = 1; j < nc; ++j) if (z[j] > mx) mx = z[j];
        double se = 0.0;
        for (int j = 0; j < nc; ++j) se += exp(z[j] - mx);
        loss += log(se) + mx - z[label[s]];
        for (int j = 0; j < nc; ++j) dz[j] = exp(z[j] - mx) / se - (j == label[s] ? 1.0 : 0.0);
        double r = z[nc] - log_stop[s];
        double ar = fabs(r);
        loss += lambda * (ar <= delta ? 0.5 * r * r : delta * (ar - 0.5 * delta));
        dz[nc] = lambda * (ar <= delta ? r : (r > 0 ? delta : -delta));
        for (int j = 0; j < no; ++j) dz[j] /= (double)n;
        /* backward through the three layers */
        for (int j = 0; j < no; ++j) gb3[j] += dz[j];
        for (int i = 0; i < h; ++i) {
            double acc = 0.0;
            for (int j = 0; j < no; ++j) { g3[i * no + j] += h2[i] * dz[j]; acc += w3[i * no + j] * dz[j]; }
            dh2[i] = h2[i] > 0 ? acc : 0.0;
        }
        for (int j = 0; j < h; ++j) gb2[j] += dh2[j];
        for (int i = 0; i < h; ++i) {
            double acc = 0.0;
            for (int j = 0; j < h; ++j) { g2[i * h + j] += h1[i] * dh2[j]; acc += w2[i * h + j] * dh2[j]; }
            dh1[i] = h1[i] > 0 ? acc : 0.0;
        }
        for (int j = 0; j < h; ++j) gb1[j] += dh1[j];
        for (int i = 0; i < din; ++i)
            for (int j = 0; j < h; ++j) g1[i * h + j] += xs[i] * dh1[j];
    }
    free(h1); free(h2); free(z); free(dz); free(dh2); free(dh1);
    return loss / (double)n;
}

/* ------------------------------------------------------------------------ */
/* Expansion traces: the vertices each query expands, in order (at most cap
 * per query; counts receive the full number). */
int orc_search_expansions(const orc_index *ix, const float *q, int64_t nq, int L, int32_t *trace,
                          int cap, int32_t *counts)
{
    scratch_t s;
    if (scratch_init(&s, ix->n_slots, L, ix->search_width, ix->R)) return ORC_E_NOMEM;
    const int d = ix->dim, R = ix->R;
    double *qlp = malloc(sizeof(double) * d);
    for (int64_t i = 0; i < nq; ++i) {
        const float *qf = q + i * d;
        lp_vector(ix->precision, qf, d, 1, qlp);
        /* the search of search_one, recording parents */
        qstats st;
        memset(&st, 0, sizeof st);
        int E = ix->entry_samples > 0 ? ix->entry_samples : L;
        int64_t alive_n = 0;
        for (int64_t u = 0; u < ix->n_slots; ++u) alive_n += ix->alive[u];
        uint64_t key = ix->seed ^ fnv1a64((const unsigned char *)qf, (size_t)d * sizeof(float));
        int64_t want = E < alive_n ? E : alive_n;
        int ne = 0;
        for (int64_t j = 0; j < 8LL * E + 64 && ne < want; ++j) {
            int64_t id = (int64_t)(((splitmix64_out(key, (uint64_t)j) >> 32) * (uint64_t)ix->n_slots) >> 32);
            if (!ix->alive[id] || s.visited[id]) continue;
            visit(&s, (int32_t)id);
            s.fresh[ne].id = (int32_t)id;
            s.fresh[ne].d = dist(ix->metric, qlp, ix->vec_lp + id * d, d);
            s.fresh[ne].expanded = 0;
            ++ne;
        }
        qsort(s.fresh, ne, sizeof(pentry), cmp_pentry);
        int np = ne < L ? ne : L;
        memcpy(s.pool, s.fresh, np * sizeof(pentry));
        int nt = 0;
        for (;;) {
            int par[8], npar = 0;
            for (int t = 0; t < np && npar < ix->search_width; ++t) if (!s.pool[t].expanded) par[npar++] = t;
            if (npar == 0) break;
            int nf = 0;
            for (int t = 0; t < npar; ++t) {
                s.pool[par[t]].expanded = 1;
                if (nt < cap) trace[i * cap + nt] = s.pool[par[t]].id;
                ++nt;
                const int32_t *row = ix->rows + (int64_t)s.pool[par[t]].id * R;
                for (int r = 0; r < R; ++r) {
                    int32_t u = row[r];
                    if (u < 0 || u >= ix->n_slots || !ix->alive[u] || s.visited[u]) continue;
                    visit(&s, u);
                    s.fresh[nf].id = u;
                    s.fresh[nf].d = dist(ix->metric, qlp, ix->vec_lp + (int64_t)u * d, d);
                    s.fresh[nf].expanded = 0;
                    ++nf;
                }
            }
            memcpy(s.merged, s.pool, np * sizeof(pentry));
            memcpy(s.merged + np, s.fresh, nf * sizeof(pentry));
            int nm = np + nf;
            qsort(s.merged, nm, sizeof(pentry), cmp_pentry);
            np = nm < L ? nm : L;
            memcpy(s.pool, s.merged, np * sizeof(pentry));
        }
        unvisit_all(&s);
        counts[i] = nt;
    }
    free(qlp);
    scratch_free(&s);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Workload-aware vector placement (Sec. 4.3, Alg. 2, Eq. 2) replayed over
 * per-batch access traces, in the batched form:
 *   F_lambda(x) = alpha * F_recent(x) + beta * log(1 + E_in(x)).
 * Per batch: F_recent halves, then counts this batch's accesses; accesses to
 * resident vectors are hits and set the reference bit of their slot.  The
 * distinct missed vectors with F_lambda > theta, by (F_lambda desc, id asc),
 * at most `promote_max` of them, are placed one after another (Alg. 2):
 *   - into a free slot while the cache is not full (Alg. 2 covers the full
 *     cache);
 *   - else F_min = the least F_lambda over residents whose reference bit is
 *     clear; the clock hand then walks from where it stands: a slot with a
 *     set bit has it cleared and the hand moves on; the first slot with a
 *     clear bit whose vector has F_lambda = F_min is the victim.  The new
 *     vector takes that slot with a clear bit, and the hand stays on it.
 *     When every bit is set, the minimum over an empty set leaves the sweep
 *     without a target: it then goes round once clearing every bit (the hand
 *     comes back to where it started) and F_min is taken over all residents.
 * A deleted vector counts F_lambda = -1.
 * theta adaptation (Sec. 4.4), when adapt > 1: once a batch's accesses are
 * counted, its miss rate (missed accesses / accesses) and the mean F_lambda
 * of its distinct missed alive vectors (summed in id order) are compared
 * with those of the previous batch that had accesses: if both rose, theta is
 * multiplied by adapt; if both fell, it is divided by adapt but kept at or
 * above the starting theta.  The theta in force for each batch's placements
 * is written to theta_out[b] (may be NULL).
 * With warm != 0 the cache starts warm (cold-start placement, Sec. 4.4): the
 * alive vectors of highest E_in, ties by id, fill slots 0, 1, ... in order.
 * trace: concatenated accesses, batch b spanning [off[b], off[b+1]).
 * Out: hits per batch, and the final slot -> id table (-1 empty). */
static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

void orc_wavp_replay(int64_t n, int64_t C, const int32_t *e_in, const uint8_t *alive,
                     const int32_t *trace, const int64_t *off, int nb, double alpha, double beta,
                     double theta, int promote_max, int warm, double adapt, int64_t *hits,
                     int32_t *slot_id, double *theta_out)
{
    double *fr = calloc(n > 0 ? n : 1, sizeof(double));
    int32_t *where = malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    uint8_t *ref = calloc(C > 0 ? C : 1, 1);
    uint8_t *cand_mark = calloc(n > 0 ? n : 1, 1);
    for (int64_t i = 0; i < n; ++i) where[i] = -1;
    for (int64_t s = 0; s < C; ++s) slot_id[s] = -1;
    int64_t used = 0, clock = 0;
    const double theta0 = theta;
    int have_prev = 0;
    int64_t prev_miss = 0, prev_acc = 0;
    double prev_mean = 0.0;
    if (warm) {
        /* repeatedly take the best remaining alive vector by (E_in desc, id asc) */
        uint8_t *taken = calloc(n > 0 ? n : 1, 1);
        while (used < C) {
            int64_t best = -1;
            for (int64_t x = 0; x < n; ++x) {
                if (!alive[x] || taken[x]) continue;
                if (best < 0 || e_in[x] > e_in[best]) best = x;
            }
            if (best < 0) break;
            taken[best] = 1;
            slot_id[used] = (int32_t)best; where[best] = (int32_t)used; ++used;
        }
        free(taken);
    }
    typedef struct { double f; int32_t id; } cand_t;
    int64_t maxlen = 0;
    for (int b = 0; b < nb; ++b) if (off[b + 1] - off[b] > maxlen) maxlen = off[b + 1] - off[b];
    cand_t *cand = malloc(sizeof(cand_t) * (maxlen + 1));
    int32_t *missed = malloc(sizeof(int32_t) * (maxlen + 1));
#define FLAM(x) (alive[(x)] ? alpha * fr[(x)] + beta * log(1.0 + (double)e_in[(x)]) : -1.0)
    for (int b = 0; b < nb; ++b) {
        for (int64_t i = 0; i < n; ++i) fr[i] *= 0.5;
        int64_t h = 0;
        for (int64_t t = off[b]; t < off[b + 1]; ++t) {
            int32_t x = trace[t];
            fr[x] += 1.0;
            if (where[x] >= 0) { ++h; ref[where[x]] = 1; }
        }
        hits[b] = h;
        /* the distinct missed vectors of the batch */
        int nm = 0;
        for (int64_t t = off[b]; t < off[b + 1]; ++t) {
            int32_t x = trace[t];
            if (where[x] >= 0 || cand_mark[x]) continue;
            cand_mark[x] = 1;
            missed[nm++] = x;
        }
        for (int i = 0; i < nm; ++i) cand_mark[missed[i]] = 0;
        qsort(missed, nm, sizeof(int32_t), cmp_i32);
        /* theta adaptation from the batch's miss rate and mean prediction */
        const int64_t acc = off[b + 1] - off[b], miss = acc - h;
        if (adapt > 1.0 && acc > 0) {
            double sum = 0.0;
            int64_t cnt = 0;
            for (int i = 0; i < nm; ++i)
                if (alive[missed[i]]) { sum += FLAM(missed[i]); ++cnt; }
            const double mean = cnt ? sum / (double)cnt : 0.0;
            if (have_prev) {
                /* miss / acc against prev_miss / prev_acc, exactly */
                const int rose = miss * prev_acc > prev_miss * acc;
                const int fell = miss * prev_acc < prev_miss * acc;
                if (rose && mean > prev_mean) theta *= adapt;
                else if (fell && mean < prev_mean) {
                    theta /= adapt;
                    if (theta < theta0) theta = theta0;
                }
            }
            have_prev = 1; prev_miss = miss; prev_acc = acc; prev_mean = mean;
        }
        if (theta_out) theta_out[b] = theta;
        int nc = 0;
        for (int i = 0; i < nm; ++i) {
            double f = FLAM(missed[i]);
            if (f > theta) { cand[nc].f = f; cand[nc].id = missed[i]; ++nc; }
        }
        /* order: F_lambda descending, id ascending */
        for (int i = 1; i < nc; ++i) {
            cand_t c = cand[i];
            int j = i - 1;
            while (j >= 0 && (cand[j].f < c.f || (cand[j].f == c.f && cand[j].id > c.id))) {
                cand[j + 1] = cand[j];
                --j;
            }
            cand[j + 1] = c;
        }
        if (nc > promote_max) nc = promote_max;
        for (int i = 0; i < nc; ++i) {
            int32_t x = cand[i].id;
            if (used < C) {
                slot_id[used] = x; where[x] = (int32_t)used; ref[used] = 0; ++used;
                continue;
            }
            if (C == 0) break;
            /* F_min over residents with a clear reference bit */
            int any = 0;
            double fmin = 0.0;
            for (int64_t s = 0; s < C; ++s)
                if (!ref[s] && (!any || FLAM(slot_id[s]) < fmin)) { fmin = FLAM(slot_id[s]); any = 1; }
            if (!any) {
                /* every bit set: one full round clears them all */
                for (int64_t s = 0; s < C; ++s) ref[s] = 0;
                for (int64_t s = 0; s < C; ++s)
                    if (s == 0 || FLAM(slot_id[s]) < fmin) fmin = FLAM(slot_id[s]);
            }
            for (;;) {
                const int64_t s = clock;
                if (!ref[s] && FLAM(slot_id[s]) == fmin) {
                    where[slot_id[s]] = -1;
                    slot_id[s] = x; where[x] = (int32_t)s; ref[s] = 0;
                    break;
                }
                if (ref[s]) ref[s] = 0;
                clock = (clock + 1) % C;
            }
        }
    }
#undef FLAM
    free(fr); free(where); free(ref); free(cand_mark); free(cand); free(missed);
}

/* ------------------------------------------------------------------------ */
/* The classic replacement policies the paper compares WAVP with (Sec. 6,
 * replacement strategies), in the same batched form over the same traces:
 *   LRU (policy 1): score = last access, ordered by (batch, position in the
 *     batch's trace); vectors never accessed (a warm start) tie at the bottom;
 *   LFU (policy 2): score = number of accesses so far;
 *   LRFU (policy 3): score = F_recent, the access count halved once per
 *     batch (combined recency and frequency with one halving per batch).
 * Per batch: accesses are counted (hits as for WAVP); the distinct missed
 * vertices, best score first (ties by id), at most promote_max of them, are
 * each placed into a free slot or in place of the resident vertex of lowest
 * score (ties by id), which is always evicted.  warm: as in orc_wavp_replay. */
void orc_policy_replay(int policy, int64_t n, int64_t C, const int32_t *e_in, const uint8_t *alive,
                       const int32_t *trace, const int64_t *off, int nb, int promote_max, int warm,
                       int64_t *hits, int32_t *slot_id)
{
    double *fr = calloc(n > 0 ? n : 1, sizeof(double));
    int64_t *freq = calloc(n > 0 ? n : 1, sizeof(int64_t));
    int64_t *last = malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    int32_t *where = malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    uint8_t *mark = calloc(n > 0 ? n : 1, 1);
    for (int64_t i = 0; i < n; ++i) { where[i] = -1; last[i] = -1; }
    for (int64_t s = 0; s < C; ++s) slot_id[s] = -1;
    int64_t used = 0;
    if (warm) {
        uint8_t *taken = calloc(n > 0 ? n : 1, 1);
        while (used < C) {
            int64_t best = -1;
            for (int64_t x = 0; x < n; ++x) {
                if (!alive[x] || taken[x]) continue;
                if (best < 0 || e_in[x] > e_in[best]) best = x;
            }
            if (best < 0) break;
            taken[best] = 1;
            slot_id[used] = (int32_t)best; where[best] = (int32_t)used; ++used;
        }
        free(taken);
    }
    int64_t maxlen = 0;
    for (int b = 0; b < nb; ++b) if (off[b + 1] - off[b] > maxlen) maxlen = off[b + 1] - off[b];
    int32_t *cand = malloc(sizeof(int32_t) * (maxlen + 1));
    /* a < b in the policy's order of importance (a less important) */
#define SCORE_LESS(a, b) \
    (policy == 1 ? (last[(a)] < last[(b)] || (last[(a)] == last[(b)] && (a) > (b))) : \
     policy == 2 ? (freq[(a)] < freq[(b)] || (freq[(a)] == freq[(b)] && (a) > (b))) : \
                   (fr[(a)] < fr[(b)] || (fr[(a)] == fr[(b)] && (a) > (b))))
    for (int b = 0; b < nb; ++b) {
        for (int64_t i = 0; i < n; ++i) fr[i] *= 0.5;
        int64_t h = 0;
        for (int64_t t = off[b]; t < off[b + 1]; ++t) {
            int32_t x = trace[t];
            fr[x] += 1.0;
            freq[x] += 1;
            last[x] = ((int64_t)b << 40) + (t - off[b]);
            if (where[x] >= 0) ++h;
        }
        hits[b] = h;
        int nc = 0;
        for (int64_t t = off[b]; t < off[b + 1]; ++t) {
            int32_t x = trace[t];
            if (where[x] >= 0 || mark[x]) continue;
            mark[x] = 1;
            cand[nc++] = x;
        }
        for (int i = 0; i < nc; ++i) mark[cand[i]] = 0;
        /* most important first */
        for (int i = 1; i < nc; ++i) {
            int32_t c = cand[i];
            int j = i - 1;
            while (j >= 0 && SCORE_LESS(cand[j], c)) { cand[j + 1] = cand[j]; --j; }
            cand[j + 1] = c;
        }
        if (nc > promote_max) nc = promote_max;
        for (int i = 0; i < nc; ++i) {
            int32_t x = cand[i];
            if (used < C) { slot_id[used] = x; where[x] = (int32_t)used; ++used; continue; }
            if (C == 0) break;
            int64_t vs = 0;
            for (int64_t s2 = 1; s2 < C; ++s2)
                if (SCORE_LESS(slot_id[s2], slot_id[vs])) vs = s2;
            where[slot_id[vs]] = -1;
            slot_id[vs] = x; where[x] = (int32_t)vs;
        }
    }
#undef SCORE_LESS
    free(fr); free(freq); free(last); free(where); free(mark); free(cand);
}
