/*
 * Seeded synthetic inputs shared by the oracle tests and the GPU path.
 *
 * This module holds no arithmetic of the SpMM method: it only draws random
 * numbers and arranges them into inputs (a CSR graph, dense matrices, edge
 * weights).  Both sides receive the same arrays from here.
 *
 * Random numbers: a counter-based SplitMix64 stream (Steele, Lea and Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014).  The i-th
 * draw of a stream keyed by K is mix64(K + (i + 1) * golden_gamma), so any
 * draw can be computed independently of the others, in any thread order.
 *
 * Graphs: the R-MAT recursive model (Chakrabarti, Zhan and Faloutsos, SDM
 * 2004) with the quadrant probabilities the paper uses in its evaluation
 * (a = 0.57, b = 0.19, c = 0.19, d = 0.05).  Each sample descends `scale`
 * levels; at every level one 32-bit draw picks a quadrant against integer
 * thresholds floor(a 2^32), floor((a+b) 2^32), floor((a+b+c) 2^32).
 * Sample (u, v) is the edge u -> v, stored at A[u][v] (row = source).
 * Self-loops are dropped, the graph is optionally symmetrised (A | A^T) and
 * duplicates are removed, giving a binary CSR with sorted unique columns.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* Progress lines on stderr while a large graph is built (0 = silent). */
static int g_verbose = 0;
void synth_set_verbose(int v) { g_verbose = v; }
static void note(const char* what, int64_t done, int64_t total) {
    if (g_verbose) {
        fprintf(stderr, "[synth] %s: %lld / %lld\n", what, (long long)done, (long long)total);
        fflush(stderr);
    }
}

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Key of stream `stream` under user seed `seed`. */
uint64_t synth_stream_key(uint64_t seed, uint64_t stream) {
    return mix64(mix64(seed + GOLDEN) + stream * 0xD1B54A32D192ED03ULL);
}

/* The ctr-th 64-bit draw of the stream keyed by key. */
static inline uint64_t draw(uint64_t key, uint64_t ctr) {
    return mix64(key + (ctr + 1) * GOLDEN);
}

uint64_t synth_draw(uint64_t key, uint64_t ctr) { return draw(key, ctr); }

enum { STREAM_RMAT = 1, STREAM_XUNIF = 2, STREAM_XINT = 3, STREAM_WEIGHT = 4, STREAM_SBM = 5, STREAM_PERM = 6 };
enum { KIND_RMAT = 0, KIND_SBM = 1 };

/* ---------------------------------------------------------------- R-MAT */

typedef struct {
    int scale;
    int64_t n, nsamples, nnz;
    int symmetrize;
    uint64_t key;
    uint32_t ta, tab, tabc;
    int64_t* off;     /* [n+1] bucket offsets                */
    uint32_t* cnt;    /* [n]   unique entries per row        */
    uint32_t* bucket; /* [off[n]] sorted/deduped per row     */
    int kind;         /* KIND_RMAT or KIND_SBM               */
    int64_t clusters; /* SBM: clusters [k n / c, (k+1) n / c) */
    uint32_t p_in;    /* SBM: P(edge drawn inside) * 2^32    */
    uint32_t* perm;   /* SBM: vertex relabelling, or NULL    */
} synth_graph;

static inline void rmat_sample(const synth_graph* g, uint64_t e, uint32_t* u, uint32_t* v) {
    uint32_t r = 0, c = 0;
    const int words = (g->scale + 1) / 2;
    for (int w = 0; w < words; ++w) {
        uint64_t z = draw(g->key, (uint64_t)e * (uint64_t)words + (uint64_t)w);
        for (int half = 0; half < 2; ++half) {
            int lvl = 2 * w + half;
            if (lvl >= g->scale) break;
            uint32_t x = half == 0 ? (uint32_t)(z >> 32) : (uint32_t)z;
            uint32_t rb = x >= g->tab;
            uint32_t cb = (x >= g->ta && x < g->tab) || x >= g->tabc;
            r = (r << 1) | rb;
            c = (c << 1) | cb;
        }
    }
    *u = r;
    *v = c;
}

/* Uniform integer in [0, m) from the high 32 bits of z (m < 2^32). */
static inline uint32_t below(uint64_t z, uint64_t m) { return (uint32_t)(((z >> 32) * m) >> 32); }

/* Stochastic block model sample e: u uniform; with probability p_in, v
   uniform in u's cluster, else v uniform over all vertices; then both are
   relabelled by perm when the graph is unclustered. */
static inline void sbm_sample(const synth_graph* g, uint64_t e, uint32_t* u, uint32_t* v) {
    const uint64_t n = (uint64_t)g->n, c = (uint64_t)g->clusters;
    const uint64_t z0 = draw(g->key, 3 * e), z1 = draw(g->key, 3 * e + 1), z2 = draw(g->key, 3 * e + 2);
    uint32_t a = below(z0, n), b;
    if ((uint32_t)(z1 >> 32) < g->p_in) {
        const uint64_t k = (uint64_t)a * c / n;                      /* a's cluster */
        const uint64_t lo = k * n / c, hi = (k + 1) * n / c;
        b = (uint32_t)(lo + below(z2, hi - lo));
    } else {
        b = below(z2, n);
    }
    if (g->perm) { a = g->perm[a]; b = g->perm[b]; }
    *u = a;
    *v = b;
}

static inline void graph_sample(const synth_graph* g, uint64_t e, uint32_t* u, uint32_t* v) {
    if (g->kind == KIND_SBM) sbm_sample(g, e, u, v);
    else rmat_sample(g, e, u, v);
}

static void sort_u32(uint32_t* a, int64_t n) {
    while (n > 24) {
        uint32_t x = a[0], y = a[n / 2], z = a[n - 1], p;
        if (x < y) p = (y < z) ? y : ((x < z) ? z : x);
        else p = (x < z) ? x : ((y < z) ? z : y);
        int64_t i = -1, j = n;
        for (;;) {
            do ++i; while (a[i] < p);
            do --j; while (a[j] > p);
            if (i >= j) break;
            uint32_t t = a[i]; a[i] = a[j]; a[j] = t;
        }
        int64_t left = j + 1;
        if (left < n - left) { sort_u32(a, left); a += left; n -= left; }
        else { sort_u32(a + left, n - left); n = left; }
    }
    for (int64_t i = 1; i < n; ++i) {
        uint32_t t = a[i];
        int64_t j = i - 1;
        while (j >= 0 && a[j] > t) { a[j + 1] = a[j]; --j; }
        a[j + 1] = t;
    }
}

static void exclusive_scan_u32_to_i64(const uint32_t* in, int64_t* out, int64_t n) {
    int nt = omp_get_max_threads();
    int64_t* part = (int64_t*)calloc((size_t)nt + 1, sizeof(int64_t));
    #pragma omp parallel num_threads(nt)
    {
        int t = omp_get_thread_num(), T = omp_get_num_threads();
        int64_t lo = n * t / T, hi = n * (t + 1) / T, s = 0;
        for (int64_t i = lo; i < hi; ++i) s += in[i];
        part[t + 1] = s;
        #pragma omp barrier
        #pragma omp single
        for (int q = 1; q <= T; ++q) part[q] += part[q - 1];
        s = part[t];
        for (int64_t i = lo; i < hi; ++i) { out[i] = s; s += in[i]; }
        if (t == T - 1) out[n] = s;
    }
    free(part);
}

/* Draw the samples of g (n, nsamples, symmetrize and the generator fields
   set), bucket them by row, sort and deduplicate each row.  Returns 0, or
   -1 on allocation failure (g is then freed). */
static int graph_build(synth_graph* g, synth_graph** out, int64_t* n_out, int64_t* nnz_out) {
    const int64_t n = g->n, nsamples = g->nsamples;
    const int symmetrize = g->symmetrize;
    g->cnt = (uint32_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(uint32_t));
    g->off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!g->cnt || !g->off) goto fail;

    /* pass 1: per-row sample counts (in eight chunks, for progress lines) */
    for (int64_t c = 0; c < 8; ++c) {
        const int64_t e0 = nsamples * c / 8, e1 = nsamples * (c + 1) / 8;
        #pragma omp parallel for schedule(static, 65536)
        for (int64_t e = e0; e < e1; ++e) {
            uint32_t u, v;
            graph_sample(g, (uint64_t)e, &u, &v);
            if (u == v) continue;
            __atomic_fetch_add(&g->cnt[u], 1u, __ATOMIC_RELAXED);
            if (symmetrize) __atomic_fetch_add(&g->cnt[v], 1u, __ATOMIC_RELAXED);
        }
        note("samples counted", e1, nsamples);
    }
    exclusive_scan_u32_to_i64(g->cnt, g->off, n);
    g->bucket = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(g->off[n] > 0 ? g->off[n] : 1));
    if (!g->bucket) goto fail;
    memset(g->cnt, 0, sizeof(uint32_t) * (size_t)n);

    /* pass 2: scatter samples into their row buckets (same draws again) */
    for (int64_t c = 0; c < 8; ++c) {
        const int64_t e0 = nsamples * c / 8, e1 = nsamples * (c + 1) / 8;
        #pragma omp parallel for schedule(static, 65536)
        for (int64_t e = e0; e < e1; ++e) {
            uint32_t u, v;
            graph_sample(g, (uint64_t)e, &u, &v);
            if (u == v) continue;
            uint32_t p = __atomic_fetch_add(&g->cnt[u], 1u, __ATOMIC_RELAXED);
            g->bucket[g->off[u] + p] = v;
            if (symmetrize) {
                uint32_t q = __atomic_fetch_add(&g->cnt[v], 1u, __ATOMIC_RELAXED);
                g->bucket[g->off[v] + q] = u;
            }
        }
        note("samples bucketed", e1, nsamples);
    }

    /* pass 3: sort each row, drop duplicates; cnt[u] becomes the unique count */
    int64_t nnz = 0;
    #pragma omp parallel for schedule(dynamic, 512) reduction(+ : nnz)
    for (int64_t u = 0; u < n; ++u) {
        uint32_t* r = g->bucket + g->off[u];
        int64_t m = g->off[u + 1] - g->off[u];
        if (m == 0) { g->cnt[u] = 0; continue; }
        sort_u32(r, m);
        int64_t w = 1;
        for (int64_t i = 1; i < m; ++i)
            if (r[i] != r[w - 1]) r[w++] = r[i];
        g->cnt[u] = (uint32_t)w;
        nnz += w;
    }
    note("rows sorted and deduplicated", n, n);
    g->nnz = nnz;
    *out = g;
    *n_out = n;
    *nnz_out = nnz;
    return 0;
fail:
    free(g->cnt); free(g->off); free(g->bucket); free(g->perm); free(g);
    return -1;
}

/*
 * Generate an R-MAT graph: nsamples edge samples at the given scale.
 * On success *out holds the sorted, deduplicated adjacency lists; call
 * synth_rmat_finish to copy them into caller-owned CSR arrays.
 * Returns 0 on success, -1 on allocation failure.
 */
int synth_rmat_begin(int scale, int64_t nsamples, double a, double b, double c,
                     uint64_t seed, int symmetrize, synth_graph** out,
                     int64_t* n_out, int64_t* nnz_out) {
    if (scale < 1 || scale > 31 || nsamples < 0) return -1;
    synth_graph* g = (synth_graph*)calloc(1, sizeof(synth_graph));
    if (!g) return -1;
    g->kind = KIND_RMAT;
    g->scale = scale;
    g->n = (int64_t)1 << scale;
    g->nsamples = nsamples;
    g->symmetrize = symmetrize;
    g->key = synth_stream_key(seed, STREAM_RMAT);
    g->ta = (uint32_t)floor(a * 4294967296.0);
    g->tab = (uint32_t)floor((a + b) * 4294967296.0);
    g->tabc = (uint32_t)floor((a + b + c) * 4294967296.0);
    return graph_build(g, out, n_out, nnz_out);
}

/* Vertex relabelling of an unclustered SBM graph: a Fisher-Yates shuffle of
   0..n-1 driven by the PERM stream of seed. */
void synth_sbm_perm(int64_t n, uint64_t seed, uint32_t* perm) {
    const uint64_t key = synth_stream_key(seed, STREAM_PERM);
    for (int64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {
        const int64_t j = (int64_t)below(draw(key, (uint64_t)i), (uint64_t)(i + 1));
        uint32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
}

/*
 * Generate a stochastic block model graph: n vertices in `clusters` equal
 * contiguous ranges, nsamples edge samples, each drawn inside its source's
 * cluster with probability p_in, else uniformly; with clustered = 0 the
 * vertices are relabelled by synth_sbm_perm(n, seed).  Self-loops and
 * duplicates are removed.  Same contract as synth_rmat_begin.
 */
int synth_sbm_begin(int64_t n, int64_t clusters, int64_t nsamples, double p_in, int clustered, uint64_t seed,
                    int symmetrize, synth_graph** out, int64_t* n_out, int64_t* nnz_out) {
    if (n < 1 || n >= ((int64_t)1 << 31) || clusters < 1 || clusters > n || nsamples < 0 ||
        !(p_in >= 0.0 && p_in <= 1.0))
        return -1;
    synth_graph* g = (synth_graph*)calloc(1, sizeof(synth_graph));
    if (!g) return -1;
    g->kind = KIND_SBM;
    g->n = n;
    g->nsamples = nsamples;
    g->symmetrize = symmetrize;
    g->clusters = clusters;
    g->p_in = p_in >= 1.0 ? 0xFFFFFFFFu : (uint32_t)floor(p_in * 4294967296.0);
    g->key = synth_stream_key(seed, STREAM_SBM);
    if (!clustered) {
        g->perm = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
        if (!g->perm) { free(g); return -1; }
        synth_sbm_perm(n, seed, g->perm);
    }
    return graph_build(g, out, n_out, nnz_out);
}

/* Raw SBM samples (before self-loop removal and dedup), for generator tests. */
void synth_sbm_samples(int64_t n, int64_t clusters, int64_t e0, int64_t count, double p_in, uint64_t seed,
                       uint32_t* u, uint32_t* v) {
    synth_graph g;
    memset(&g, 0, sizeof g);
    g.kind = KIND_SBM;
    g.n = n;
    g.clusters = clusters;
    g.p_in = p_in >= 1.0 ? 0xFFFFFFFFu : (uint32_t)floor(p_in * 4294967296.0);
    g.key = synth_stream_key(seed, STREAM_SBM);
    #pragma omp parallel for schedule(static, 65536)
    for (int64_t i = 0; i < count; ++i) sbm_sample(&g, (uint64_t)(e0 + i), &u[i], &v[i]);
}

/* Copy the graph into caller-owned row_ptr[n+1] / col[nnz] and free it. */
void synth_rmat_finish(synth_graph* g, int64_t* row_ptr, int32_t* col) {
    const int64_t n = g->n;
    exclusive_scan_u32_to_i64(g->cnt, row_ptr, n);
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t u = 0; u < n; ++u)
        memcpy(col + row_ptr[u], g->bucket + g->off[u], sizeof(uint32_t) * g->cnt[u]);
    free(g->cnt); free(g->off); free(g->bucket); free(g->perm); free(g);
}

void synth_rmat_free(synth_graph* g) {
    if (!g) return;
    free(g->cnt); free(g->off); free(g->bucket); free(g->perm); free(g);
}

/* Raw samples (before self-loop removal and dedup), for generator tests. */
void synth_rmat_samples(int scale, int64_t e0, int64_t count, double a, double b, double c,
                        uint64_t seed, uint32_t* u, uint32_t* v) {
    synth_graph g;
    memset(&g, 0, sizeof g);
    g.scale = scale;
    g.key = synth_stream_key(seed, STREAM_RMAT);
    g.ta = (uint32_t)floor(a * 4294967296.0);
    g.tab = (uint32_t)floor((a + b) * 4294967296.0);
    g.tabc = (uint32_t)floor((a + b + c) * 4294967296.0);
    #pragma omp parallel for schedule(static, 65536)
    for (int64_t i = 0; i < count; ++i) rmat_sample(&g, (uint64_t)(e0 + i), &u[i], &v[i]);
}

/* ------------------------------------------------------- dense matrices */

/* X[i*ld + j] = (draw >> 40) * 2^-24: uniform on [0,1), exact in FP32. */
void synth_uniform(int64_t n, int64_t k, int64_t ld, uint64_t seed, float* X) {
    const uint64_t key = synth_stream_key(seed, STREAM_XUNIF);
    #pragma omp parallel for schedule(static, 16384)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < k; ++j)
            X[i * ld + j] = (float)(draw(key, (uint64_t)(i * k + j)) >> 40) * 0x1p-24f;
}

/* X[i*ld + j] = draw >> 61: integers in {0..7}. */
void synth_int07(int64_t n, int64_t k, int64_t ld, uint64_t seed, float* X) {
    const uint64_t key = synth_stream_key(seed, STREAM_XINT);
    #pragma omp parallel for schedule(static, 16384)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < k; ++j)
            X[i * ld + j] = (float)(draw(key, (uint64_t)(i * k + j)) >> 61);
}

/*
 * Lognormal(0,1) edge weights, keyed by the unordered pair {u, v} so that a
 * symmetric pattern gets symmetric values: z by Box-Muller in FP64 from two
 * uniforms on (0,1], val = (float)exp(z).
 */
void synth_lognormal_weights(int64_t n, const int64_t* row_ptr, const int32_t* col,
                             uint64_t seed, float* val) {
    const uint64_t key = synth_stream_key(seed, STREAM_WEIGHT);
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t u = 0; u < n; ++u)
        for (int64_t p = row_ptr[u]; p < row_ptr[u + 1]; ++p) {
            uint64_t v = (uint64_t)(uint32_t)col[p];
            uint64_t lo = (uint64_t)u < v ? (uint64_t)u : v, hi = (uint64_t)u < v ? v : (uint64_t)u;
            uint64_t pk = mix64((lo << 32) ^ hi ^ key);
            double u1 = ((double)(draw(pk, 0) >> 11) + 1.0) * 0x1p-53;
            double u2 = (double)(draw(pk, 1) >> 11) * 0x1p-53;
            double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
            val[p] = (float)exp(z);
        }
}

/* out[i] = draw(key, ctr0 + i) for i < count. */
void synth_draws(uint64_t key, uint64_t ctr0, int64_t count, uint64_t* out) {
    for (int64_t i = 0; i < count; ++i) out[i] = draw(key, ctr0 + (uint64_t)i);
}
