/*
 * Seeded synthetic graph inputs: Kronecker (R-MAT) and Erdos-Renyi graphs in CSR
 * form, plus seeded root selection.
 *
 * This module only produces inputs.  It holds none of the breadth-first-search
 * arithmetic; both the CPU oracle and the GPU library read the CSR it emits.
 *
 * Kronecker workload (Section 6.2 of the paper: Graph500 generator, SCALE and
 * edgefactor, initiator A=0.57 B=0.19 C=0.19 D=0.05, edges made bidirectional):
 *   - M = edgefactor * 2^SCALE edge draws.  Edge e picks one quadrant per bit
 *     level from a single uniform 32-bit draw r: r < A -> (0,0), r < A+B ->
 *     (0,1), r < A+B+C -> (1,0), else (1,1).
 *   - Vertex ids are then relabelled by a seeded uniform random permutation.
 *   - Both directions are stored; self-loops and duplicate entries are dropped;
 *     each row is sorted ascending.  Offsets are int64, columns int32.
 * Erdos-Renyi workload: m uniform unordered pairs over n vertices, same
 * symmetrise / dedup / sort treatment.
 *
 * Random numbers: the i-th output of a SplitMix64 stream (Steele, Lea, Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014), evaluated by
 * counter so the result does not depend on the number of threads.
 * Rows are filled in arbitrary order and then sorted, so the emitted CSR is a
 * pure function of (scale, edgefactor, seed) or (n, m, seed).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>
#include <stdio.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t splitmix_at(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * GOLDEN;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Independent stream per purpose: derive a key from (seed, tag). */
static inline uint64_t stream_key(uint64_t seed, uint64_t tag)
{
    return splitmix_at(seed ^ (tag * 0xD1B54A32D192ED03ULL), 0x51ED2701ULL);
}

/* Map a 64-bit draw to [0, bound) by the multiply-high method (Lemire 2019). */
static inline uint64_t bounded(uint64_t x, uint64_t bound)
{
    return (uint64_t)(((unsigned __int128)x * bound) >> 64);
}

typedef struct gg_state {
    int64_t n;
    int64_t *off;    /* n+1, row starts of the pre-dedup fill */
    int64_t *len;    /* n, row length after sort + dedup */
    int32_t *col;    /* pre-dedup column storage, rows compacted in place */
    int64_t nnz;     /* after dedup */
} gg_state;

typedef void (*edge_fn)(void *ctx, int64_t e, int32_t *u, int32_t *v);

typedef struct {
    int scale;
    uint64_t key;       /* quadrant stream */
    uint32_t t_a, t_ab, t_abc;
    const int32_t *perm;
} kron_ctx;

static void kron_edge(void *vctx, int64_t e, int32_t *pu, int32_t *pv)
{
    const kron_ctx *c = (const kron_ctx *)vctx;
    const int per = (c->scale + 1) / 2;         /* two levels per 64-bit draw */
    uint32_t row = 0, colb = 0;
    for (int j = 0; j < per; ++j) {
        uint64_t x = splitmix_at(c->key, (uint64_t)e * (uint64_t)per + (uint64_t)j);
        for (int h = 0; h < 2; ++h) {
            int lvl = 2 * j + h;
            if (lvl >= c->scale) break;
            uint32_t r = (uint32_t)(h ? (x >> 32) : (x & 0xFFFFFFFFu));
            uint32_t rb, cb;
            if (r < c->t_a)        { rb = 0; cb = 0; }
            else if (r < c->t_ab)  { rb = 0; cb = 1; }
            else if (r < c->t_abc) { rb = 1; cb = 0; }
            else                   { rb = 1; cb = 1; }
            row |= rb << lvl;
            colb |= cb << lvl;
        }
    }
    *pu = c->perm[row];
    *pv = c->perm[colb];
}

typedef struct {
    int64_t n;
    uint64_t key;
} er_ctx;

static void er_edge(void *vctx, int64_t e, int32_t *pu, int32_t *pv)
{
    const er_ctx *c = (const er_ctx *)vctx;
    *pu = (int32_t)bounded(splitmix_at(c->key, 2 * (uint64_t)e), (uint64_t)c->n);
    *pv = (int32_t)bounded(splitmix_at(c->key, 2 * (uint64_t)e + 1), (uint64_t)c->n);
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static void sort_i32(int32_t *a, int64_t len)
{
    if (len < 32) {                       /* insertion sort for short rows */
        for (int64_t i = 1; i < len; ++i) {
            int32_t x = a[i];
            int64_t j = i - 1;
            while (j >= 0 && a[j] > x) { a[j + 1] = a[j]; --j; }
            a[j + 1] = x;
        }
    } else {
        qsort(a, (size_t)len, sizeof(int32_t), cmp_i32);
    }
}

static void gg_free_internal(gg_state *s)
{
    if (!s) return;
    free(s->off);
    free(s->len);
    free(s->col);
    free(s);
}

/* Phase messages on stderr for long generations (gg_set_verbose). */
static int g_verbose = 0;
void gg_set_verbose(int on) { g_verbose = on; }

static void phase(const char *what, double t0)
{
    if (!g_verbose) return;
    fprintf(stderr, "[graphgen] %s done at %.1f s\n", what, omp_get_wtime() - t0);
    fflush(stderr);
}

/* Two passes over the edge stream (count, then fill), then per-row sort+dedup. */
static gg_state *build(int64_t n, int64_t m, edge_fn fn, void *ctx, int nthreads)
{
    const double t0 = omp_get_wtime();
    if (nthreads > 0) omp_set_num_threads(nthreads);
    gg_state *s = (gg_state *)calloc(1, sizeof(gg_state));
    if (!s) return NULL;
    s->n = n;
    s->off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    s->len = (int64_t *)calloc((size_t)n > 0 ? (size_t)n : 1, sizeof(int64_t));
    if (!s->off || !s->len) { gg_free_internal(s); return NULL; }
    int64_t *cnt = s->len; /* reuse as degree counter, then as cursor */

#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        int32_t u, v;
        fn(ctx, e, &u, &v);
        if (u == v) continue;
        __atomic_fetch_add(&cnt[u], 1, __ATOMIC_RELAXED);
        __atomic_fetch_add(&cnt[v], 1, __ATOMIC_RELAXED);
    }
    phase("degree count pass", t0);
    int64_t acc = 0;
    for (int64_t v = 0; v < n; ++v) { s->off[v] = acc; acc += cnt[v]; cnt[v] = 0; }
    s->off[n] = acc;
    s->col = (int32_t *)malloc((size_t)(acc > 0 ? acc : 1) * sizeof(int32_t));
    if (!s->col) { gg_free_internal(s); return NULL; }

#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        int32_t u, v;
        fn(ctx, e, &u, &v);
        if (u == v) continue;
        int64_t pu = __atomic_fetch_add(&cnt[u], 1, __ATOMIC_RELAXED);
        int64_t pv = __atomic_fetch_add(&cnt[v], 1, __ATOMIC_RELAXED);
        s->col[s->off[u] + pu] = v;
        s->col[s->off[v] + pv] = u;
    }

    phase("fill pass", t0);
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : total)
    for (int64_t v = 0; v < n; ++v) {
        int32_t *row = s->col + s->off[v];
        int64_t len = s->off[v + 1] - s->off[v];
        sort_i32(row, len);
        int64_t k = 0;
        for (int64_t i = 0; i < len; ++i)
            if (k == 0 || row[i] != row[k - 1]) row[k++] = row[i];
        s->len[v] = k;
        total += k;
    }
    s->nnz = total;
    phase("row sort and dedup", t0);
    return s;
}

static int32_t *make_perm(int64_t n, uint64_t seed)
{
    int32_t *p = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!p) return NULL;
    for (int64_t i = 0; i < n; ++i) p[i] = (int32_t)i;
    uint64_t key = stream_key(seed, 2);
    for (int64_t i = n - 1; i > 0; --i) {             /* Fisher-Yates */
        int64_t j = (int64_t)bounded(splitmix_at(key, (uint64_t)i), (uint64_t)i + 1);
        int32_t t = p[i]; p[i] = p[j]; p[j] = t;
    }
    return p;
}

gg_state *gg_kronecker(int scale, int edgefactor, uint64_t seed,
                       double a, double b, double c, int nthreads)
{
    if (scale < 0 || scale > 30 || edgefactor < 0) return NULL;
    int64_t n = (int64_t)1 << scale;
    int64_t m = (int64_t)edgefactor * n;
    kron_ctx ctx;
    ctx.scale = scale;
    ctx.key = stream_key(seed, 1);
    ctx.t_a = (uint32_t)(a * 4294967296.0);
    ctx.t_ab = (uint32_t)((a + b) * 4294967296.0);
    ctx.t_abc = (uint32_t)((a + b + c) * 4294967296.0);
    int32_t *perm = make_perm(n, seed);
    if (!perm) return NULL;
    ctx.perm = perm;
    gg_state *s = build(n, m, kron_edge, &ctx, nthreads);
    free(perm);
    return s;
}

gg_state *gg_erdos_renyi(int64_t n, int64_t m_pairs, uint64_t seed, int nthreads)
{
    if (n <= 0 || n > 0x7FFFFFFFLL || m_pairs < 0) return NULL;
    er_ctx ctx;
    ctx.n = n;
    ctx.key = stream_key(seed, 3);
    return build(n, m_pairs, er_edge, &ctx, nthreads);
}

int64_t gg_num_vertices(const gg_state *s) { return s ? s->n : -1; }
int64_t gg_nnz(const gg_state *s) { return s ? s->nnz : -1; }

/* Write the deduplicated CSR into caller arrays: off[n+1] (int64), col[nnz] (int32). */
int gg_emit(const gg_state *s, int64_t *off, int32_t *col, int nthreads)
{
    if (!s || !off || (!col && s->nnz > 0)) return -1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int64_t acc = 0;
    for (int64_t v = 0; v < s->n; ++v) { off[v] = acc; acc += s->len[v]; }
    off[s->n] = acc;
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t v = 0; v < s->n; ++v)
        memcpy(col + off[v], s->col + s->off[v], (size_t)s->len[v] * sizeof(int32_t));
    return 0;
}

void gg_free(gg_state *s) { gg_free_internal(s); }

/*
 * Draw k distinct roots uniformly from the vertices of nonzero degree
 * (a partial Fisher-Yates over the candidate list).  Returns the number drawn
 * (min(k, #candidates)).
 */
int64_t gg_pick_roots(int64_t n, const int64_t *off, uint64_t seed, int64_t k, int32_t *out)
{
    int64_t nc = 0;
    for (int64_t v = 0; v < n; ++v) nc += (off[v + 1] > off[v]);
    if (nc == 0 || k <= 0) return 0;
    int32_t *cand = (int32_t *)malloc((size_t)nc * sizeof(int32_t));
    if (!cand) return -1;
    nc = 0;
    for (int64_t v = 0; v < n; ++v)
        if (off[v + 1] > off[v]) cand[nc++] = (int32_t)v;
    if (k > nc) k = nc;
    uint64_t key = stream_key(seed, 4);
    for (int64_t i = 0; i < k; ++i) {
        int64_t j = i + (int64_t)bounded(splitmix_at(key, (uint64_t)i), (uint64_t)(nc - i));
        int32_t t = cand[i]; cand[i] = cand[j]; cand[j] = t;
        out[i] = cand[i];
    }
    free(cand);
    return k;
}

/* Uniform 64-bit draws of an independent stream (used for Poisson arrivals). */
void gg_uniform_u64(uint64_t seed, uint64_t tag, int64_t count, uint64_t *out)
{
    uint64_t key = stream_key(seed, 16 + tag);
    for (int64_t i = 0; i < count; ++i) out[i] = splitmix_at(key, (uint64_t)i);
}
