/*
 * Seeded synthetic graph generators -> CSR (row_ptr uint64, col uint32/uint64,
 * optional uint32 weights).  This module only produces inputs; it holds none
 * of the traversal arithmetic and is shared by the tests, the bench and the
 * oracle checks alike.
 *
 * Random numbers: SplitMix64 (Steele, Lea & Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) used counter-style: the n-th
 * draw of stream key k is mix64(k + (n + 1) * GAMMA), so every sample is a
 * pure function of (seed, stream, index) and the output does not depend on
 * the thread count.
 *
 * Kinds
 *   R-MAT / Kronecker (Chakrabarti, Zhan & Faloutsos, SDM 2004): m = ef * 2^scale
 *     samples, each of `scale` bit levels picks quadrant (row bit, col bit)
 *     = (0,0) w.p. a, (0,1) w.p. b, (1,0) w.p. c, (1,1) w.p. d, no noise;
 *     then vertex ids go through a keyed bijection (a Feistel network with
 *     cycle walking) so id order carries no locality.
 *   uniform: m samples with both endpoints uniform on [0, 2^scale).
 *   Chung-Lu power law: expected degree of vertex i proportional to
 *     (i + i0)^(-1/(gamma-1)); m samples, each endpoint drawn from that
 *     distribution with Vose's alias method (one draw per endpoint).
 * Every kind is then symmetrised, self-loops and duplicates dropped, and each
 * neighbour list sorted ascending.
 * Weights: w(u,v) = 1 + (mix64(wkey ^ (min(u,v) << 32 | max(u,v))) mod 255),
 * symmetric per undirected pair, uniform on [1, 255].
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>
#include <stdio.h>

#define GAMMA 0x9E3779B97F4A7C15ull

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t gg_stream_key(uint64_t seed, uint64_t stream)
{
    return mix64(mix64(seed + GAMMA) ^ (stream * GAMMA + 0x632BE59BD9B4E019ull));
}

static inline uint64_t draw(uint64_t key, uint64_t n)
{
    return mix64(key + (n + 1) * GAMMA);
}

uint64_t gg_draw(uint64_t key, uint64_t n) { return draw(key, n); }

enum { STREAM_EDGES = 1, STREAM_PERM = 2, STREAM_WEIGHT = 3 };
enum { GG_RMAT = 0, GG_UNIFORM = 1, GG_CHUNGLU = 2 };

/* ---- keyed bijection on [0, n) with n <= 2^(2h): Feistel + cycle walk ---- */
typedef struct { uint64_t key[4]; int h; uint64_t n; } perm_t;

static void perm_init(perm_t *p, uint64_t seed, uint64_t n)
{
    int bits = 1;
    while (bits < 64 && (1ull << bits) < n) ++bits;
    p->h = (bits + 1) / 2;
    p->n = n;
    for (int r = 0; r < 4; ++r) p->key[r] = draw(gg_stream_key(seed, STREAM_PERM), (uint64_t)r);
}

static inline uint64_t feistel(const perm_t *p, uint64_t x)
{
    uint64_t mask = (1ull << p->h) - 1;
    uint64_t L = (x >> p->h) & mask, R = x & mask;
    for (int r = 0; r < 4; ++r) {
        uint64_t F = mix64(p->key[r] ^ R) & mask;
        uint64_t t = L ^ F;
        L = R;
        R = t;
    }
    return (L << p->h) | R;
}

static inline uint64_t perm_apply(const perm_t *p, uint64_t x)
{
    do { x = feistel(p, x); } while (x >= p->n);
    return x;
}

/* ---- samplers ---- */
typedef struct {
    int kind;
    int scale;
    uint64_t V, m;
    uint64_t key;
    uint32_t ta, tab, tabc; /* R-MAT thresholds on 32-bit uniforms */
    perm_t perm;
    int permute;
    const uint32_t *alias_prob; /* Chung-Lu: alias table (Vose 1991), keep-threshold * 2^32 */
    const uint32_t *alias_idx;  /* Chung-Lu: alias of each slot */
} sampler_t;

static inline void sample_edge(const sampler_t *s, uint64_t k, uint64_t *pu, uint64_t *pv)
{
    uint64_t u = 0, v = 0;
    if (s->kind == GG_RMAT) {
        int levels = s->scale;
        uint64_t base = k * (uint64_t)((levels + 1) / 2);
        for (int b = 0; b < levels; ++b) {
            uint64_t x = draw(s->key, base + (uint64_t)(b / 2));
            uint32_t r = (b & 1) ? (uint32_t)x : (uint32_t)(x >> 32);
            /* quadrant of r: [0,a) -> (0,0), [a,a+b) -> (0,1), [a+b,a+b+c) -> (1,0), else (1,1) */
            const uint64_t ge_a = r >= s->ta, ge_ab = r >= s->tab, ge_abc = r >= s->tabc;
            u = (u << 1) | ge_ab;
            v = (v << 1) | ((ge_a ^ ge_ab) | ge_abc);
        }
        if (s->permute) {
            u = perm_apply(&s->perm, u);
            v = perm_apply(&s->perm, v);
        }
    } else if (s->kind == GG_UNIFORM) {
        uint64_t x = draw(s->key, 2 * k), y = draw(s->key, 2 * k + 1);
        u = s->scale ? x >> (64 - s->scale) : 0;
        v = s->scale ? y >> (64 - s->scale) : 0;
    } else {
        /* alias method: slot from the high half of one draw, keep-or-alias from the low half */
        for (int e = 0; e < 2; ++e) {
            const uint64_t x = draw(s->key, 2 * k + (uint64_t)e);
            const uint64_t slot = ((x >> 32) * s->V) >> 32;
            const uint64_t pick = ((uint32_t)x < s->alias_prob[slot]) ? slot : s->alias_idx[slot];
            if (e == 0) u = pick; else v = pick;
        }
        if (s->permute) {
            u = perm_apply(&s->perm, u);
            v = perm_apply(&s->perm, v);
        }
    }
    *pu = u;
    *pv = v;
}

/* ---- graph handle ---- */
typedef struct {
    uint64_t V, E;
    uint64_t *row_ptr; /* V+1: final CSR offsets */
    uint64_t *off;     /* V: where list v starts inside adj (adj may have gaps) */
    uint32_t *adj;     /* sorted unique lists, list v at adj[off[v] .. + deg(v)) */
} gg_graph;

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

/* LSD radix sort, 8-bit digits; passes whose digit is the same for every
 * element are skipped.  Falls back to qsort when the scratch buffer cannot be
 * allocated. */
static void radix_u32(uint32_t *a, uint64_t n)
{
    uint32_t *tmp = (uint32_t *)malloc(n * sizeof(uint32_t));
    if (!tmp) {
        qsort(a, n, sizeof(uint32_t), cmp_u32);
        return;
    }
    uint32_t *src = a, *dst = tmp;
    for (int shift = 0; shift < 32; shift += 8) {
        uint64_t c[257] = {0};
        for (uint64_t i = 0; i < n; ++i) c[((src[i] >> shift) & 0xFFu) + 1]++;
        if (c[((src[0] >> shift) & 0xFFu) + 1] == n) continue;
        for (int d = 0; d < 256; ++d) c[d + 1] += c[d];
        for (uint64_t i = 0; i < n; ++i) dst[c[(src[i] >> shift) & 0xFFu]++] = src[i];
        uint32_t *t = src;
        src = dst;
        dst = t;
    }
    if (src != a) memcpy(a, src, n * sizeof(uint32_t));
    free(tmp);
}

static void sort_u32(uint32_t *a, uint64_t n)
{
    if (n < 32) { /* insertion sort for short lists */
        for (uint64_t i = 1; i < n; ++i) {
            uint32_t x = a[i];
            uint64_t j = i;
            while (j > 0 && a[j - 1] > x) { a[j] = a[j - 1]; --j; }
            a[j] = x;
        }
    } else if (n < 1024) {
        qsort(a, n, sizeof(uint32_t), cmp_u32);
    } else {
        radix_u32(a, n);
    }
}

/* Builds the simple symmetric graph of the sampler's m samples.
 * 1. every thread draws a fixed contiguous range of samples and counts, per
 *    bucket of source vertices, the directed pairs it will emit (both
 *    directions, loops dropped);
 * 2. the same ranges are drawn again and each pair (src << 32 | dst) is
 *    written to its bucket's region (one write stream per bucket per thread);
 * 3. each bucket is counting-sorted by source vertex in cache, and every
 *    list is sorted and deduplicated.
 * The result does not depend on the thread count. */
static inline uint64_t bucket_of(uint64_t x, uint64_t nb, uint64_t V)
{
    return (x * nb) / V;
}

static gg_graph *build(const sampler_t *s)
{
    const uint64_t V = s->V, m = s->m;
    uint64_t nb = 1024;
    while (nb > 1 && V / nb < 64) nb >>= 1;
    const int T = omp_get_max_threads();
    gg_graph *g = (gg_graph *)calloc(1, sizeof(gg_graph));
    uint64_t *cnt = (uint64_t *)calloc((size_t)T * nb, sizeof(uint64_t));
    uint64_t *bstart = (uint64_t *)calloc(nb + 1, sizeof(uint64_t));
    uint32_t *deg = (uint32_t *)calloc(V ? V : 1, sizeof(uint32_t));
    uint64_t *off = (uint64_t *)malloc((V + 1) * sizeof(uint64_t));
    uint64_t *pairs = NULL;
    int failed = 0;
    if (!g || !cnt || !bstart || !deg || !off) goto fail;
    const int verbose = getenv("GG_VERBOSE") != NULL;
    double t0 = omp_get_wtime();

#pragma omp parallel num_threads(T)
    {
        const int t = omp_get_thread_num(), nt = omp_get_num_threads();
        uint64_t *c = cnt + (size_t)t * nb;
        const uint64_t k0 = m * (uint64_t)t / nt, k1 = m * (uint64_t)(t + 1) / nt;
        for (uint64_t k = k0; k < k1; ++k) {
            uint64_t u, v;
            sample_edge(s, k, &u, &v);
            if (u == v) continue;
            c[bucket_of(u, nb, V)]++;
            c[bucket_of(v, nb, V)]++;
        }
    }
    /* positions: bucket-major, thread-minor */
    {
        uint64_t run = 0;
        for (uint64_t b = 0; b < nb; ++b) {
            bstart[b] = run;
            for (int t = 0; t < T; ++t) {
                uint64_t x = cnt[(size_t)t * nb + b];
                cnt[(size_t)t * nb + b] = run;
                run += x;
            }
        }
        bstart[nb] = run;
    }
    if (verbose) fprintf(stderr, "[gg] count %.2fs\n", omp_get_wtime() - t0);
    pairs = (uint64_t *)malloc((bstart[nb] ? bstart[nb] : 1) * sizeof(uint64_t));
    g->adj = (uint32_t *)malloc((bstart[nb] ? bstart[nb] : 1) * sizeof(uint32_t));
    if (!pairs || !g->adj) goto fail;

#pragma omp parallel num_threads(T)
    {
        const int t = omp_get_thread_num(), nt = omp_get_num_threads();
        uint64_t *pos = cnt + (size_t)t * nb;
        const uint64_t k0 = m * (uint64_t)t / nt, k1 = m * (uint64_t)(t + 1) / nt;
        for (uint64_t k = k0; k < k1; ++k) {
            uint64_t u, v;
            sample_edge(s, k, &u, &v);
            if (u == v) continue;
            pairs[pos[bucket_of(u, nb, V)]++] = (u << 32) | v;
            pairs[pos[bucket_of(v, nb, V)]++] = (v << 32) | u;
        }
    }

    if (verbose) fprintf(stderr, "[gg] scatter %.2fs\n", omp_get_wtime() - t0);
#pragma omp parallel for schedule(dynamic, 1) num_threads(T)
    for (uint64_t b = 0; b < nb; ++b) {
        const uint64_t lo = (b * V + nb - 1) / nb, hi = ((b + 1) * V + nb - 1) / nb;
        const uint64_t nv = hi - lo, base = bstart[b], n = bstart[b + 1] - base;
        uint64_t *lstart = (uint64_t *)calloc(nv + 1, sizeof(uint64_t));
        if (!lstart) {
            __atomic_store_n(&failed, 1, __ATOMIC_RELAXED);
            continue;
        }
        for (uint64_t i = 0; i < n; ++i) lstart[(pairs[base + i] >> 32) - lo + 1]++;
        for (uint64_t x = 0; x < nv; ++x) lstart[x + 1] += lstart[x];
        for (uint64_t x = 0; x < nv; ++x) off[lo + x] = base + lstart[x];
        for (uint64_t i = 0; i < n; ++i) {
            uint64_t p = pairs[base + i];
            g->adj[base + lstart[(p >> 32) - lo]++] = (uint32_t)p;
        }
        /* lstart[x] now holds the end of list x */
        for (uint64_t x = 0; x < nv; ++x) {
            uint32_t *a = g->adj + off[lo + x];
            uint64_t len = (base + lstart[x]) - off[lo + x];
            sort_u32(a, len);
            uint64_t w = 0;
            for (uint64_t i = 0; i < len; ++i)
                if (i == 0 || a[i] != a[w - 1]) a[w++] = a[i];
            deg[lo + x] = (uint32_t)w;
        }
        free(lstart);
    }
    free(pairs);
    pairs = NULL;
    if (verbose) fprintf(stderr, "[gg] buckets %.2fs\n", omp_get_wtime() - t0);
    if (failed) goto fail;
    g->row_ptr = (uint64_t *)malloc((V + 1) * sizeof(uint64_t));
    if (!g->row_ptr) goto fail;
    g->row_ptr[0] = 0;
    for (uint64_t v = 0; v < V; ++v) g->row_ptr[v + 1] = g->row_ptr[v] + deg[v];
    g->E = g->row_ptr[V];
    g->V = V;
    g->off = off;
    free(deg);
    free(cnt);
    free(bstart);
    return g;
fail:
    if (g) { free(g->adj); free(g->row_ptr); free(g); }
    free(deg); free(off); free(pairs); free(cnt); free(bstart);
    return NULL;
}

void *gg_rmat(int scale, uint64_t edgefactor, double a, double b, double c,
              uint64_t seed, int permute)
{
    sampler_t s;
    memset(&s, 0, sizeof(s));
    s.kind = GG_RMAT;
    s.scale = scale;
    s.V = 1ull << scale;
    s.m = edgefactor << scale;
    s.key = gg_stream_key(seed, STREAM_EDGES);
    s.ta = (uint32_t)fmin(4294967295.0, floor(a * 4294967296.0));
    s.tab = (uint32_t)fmin(4294967295.0, floor((a + b) * 4294967296.0));
    s.tabc = (uint32_t)fmin(4294967295.0, floor((a + b + c) * 4294967296.0));
    s.permute = permute;
    perm_init(&s.perm, seed, s.V);
    return build(&s);
}

void *gg_uniform(int scale, uint64_t samples, uint64_t seed)
{
    sampler_t s;
    memset(&s, 0, sizeof(s));
    s.kind = GG_UNIFORM;
    s.scale = scale;
    s.V = 1ull << scale;
    s.m = samples;
    s.key = gg_stream_key(seed, STREAM_EDGES);
    return build(&s);
}

void *gg_chung_lu(uint64_t V, uint64_t samples, double gamma, double i0,
                  uint64_t seed, int permute)
{
    sampler_t s;
    memset(&s, 0, sizeof(s));
    /* Vose's alias table for weights (i + i0)^(-1/(gamma-1)) */
    double *pw = (double *)malloc(V * sizeof(double));
    uint32_t *prob = (uint32_t *)malloc(V * sizeof(uint32_t));
    uint32_t *alias = (uint32_t *)malloc(V * sizeof(uint32_t));
    uint32_t *small = (uint32_t *)malloc(V * sizeof(uint32_t));
    uint32_t *large = (uint32_t *)malloc(V * sizeof(uint32_t));
    if (!pw || !prob || !alias || !small || !large || V == 0 || V > 0xFFFFFFFFull) {
        free(pw); free(prob); free(alias); free(small); free(large);
        return NULL;
    }
    double total = 0.0, expo = -1.0 / (gamma - 1.0);
    for (uint64_t i = 0; i < V; ++i) total += (pw[i] = pow((double)i + i0, expo));
    uint64_t ns = 0, nl = 0;
    for (uint64_t i = 0; i < V; ++i) {
        pw[i] = pw[i] * (double)V / total;
        alias[i] = (uint32_t)i;
        if (pw[i] < 1.0) small[ns++] = (uint32_t)i; else large[nl++] = (uint32_t)i;
    }
    while (ns > 0 && nl > 0) {
        uint32_t l = small[--ns], gi = large[--nl];
        prob[l] = (uint32_t)fmin(4294967295.0, pw[l] * 4294967296.0);
        alias[l] = gi;
        pw[gi] = (pw[gi] + pw[l]) - 1.0;
        if (pw[gi] < 1.0) small[ns++] = gi; else large[nl++] = gi;
    }
    while (nl > 0) prob[large[--nl]] = 0xFFFFFFFFu;
    while (ns > 0) prob[small[--ns]] = 0xFFFFFFFFu;
    free(pw); free(small); free(large);
    s.kind = GG_CHUNGLU;
    s.V = V;
    s.m = samples;
    s.key = gg_stream_key(seed, STREAM_EDGES);
    s.alias_prob = prob;
    s.alias_idx = alias;
    s.permute = permute;
    perm_init(&s.perm, seed, V);
    gg_graph *g = build(&s);
    free(prob);
    free(alias);
    return g;
}

/* CSR from an explicit directed edge list (no symmetrising): used for small
 * hand-made graphs.  Lists are sorted; duplicates and loops are kept. */
void *gg_from_edges(uint64_t V, uint64_t n, const uint64_t *src, const uint64_t *dst)
{
    gg_graph *g = (gg_graph *)calloc(1, sizeof(gg_graph));
    if (!g) return NULL;
    g->V = V;
    g->E = n;
    g->row_ptr = (uint64_t *)calloc(V + 1, sizeof(uint64_t));
    g->adj = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    if (!g->row_ptr || !g->adj) { free(g->row_ptr); free(g->adj); free(g); return NULL; }
    for (uint64_t i = 0; i < n; ++i) g->row_ptr[src[i] + 1]++;
    for (uint64_t v = 0; v < V; ++v) g->row_ptr[v + 1] += g->row_ptr[v];
    uint64_t *pos = (uint64_t *)malloc((V ? V : 1) * sizeof(uint64_t));
    if (!pos) { free(g->row_ptr); free(g->adj); free(g); return NULL; }
    memcpy(pos, g->row_ptr, V * sizeof(uint64_t));
    for (uint64_t i = 0; i < n; ++i) g->adj[pos[src[i]]++] = (uint32_t)dst[i];
    free(pos);
    for (uint64_t v = 0; v < V; ++v) sort_u32(g->adj + g->row_ptr[v], g->row_ptr[v + 1] - g->row_ptr[v]);
    g->off = (uint64_t *)malloc((V ? V : 1) * sizeof(uint64_t));
    if (!g->off) { free(g->row_ptr); free(g->adj); free(g); return NULL; }
    memcpy(g->off, g->row_ptr, V * sizeof(uint64_t));
    return g;
}

uint64_t gg_num_vertices(void *h) { return ((gg_graph *)h)->V; }
uint64_t gg_num_edges(void *h) { return ((gg_graph *)h)->E; }

/* Copies the CSR into caller buffers (which may be pinned host memory).
 * col_bytes is 4 or 8; weights may be NULL. */
int gg_export(void *h, uint64_t *row_ptr, void *col, int col_bytes,
              uint32_t *weights, uint64_t weight_seed)
{
    gg_graph *g = (gg_graph *)h;
    if (col_bytes != 4 && col_bytes != 8) return -1;
    uint64_t V = g->V;
    memcpy(row_ptr, g->row_ptr, (V + 1) * sizeof(uint64_t));
    uint64_t wkey = gg_stream_key(weight_seed, STREAM_WEIGHT);
#pragma omp parallel for schedule(dynamic, 4096)
    for (uint64_t u = 0; u < V; ++u) {
        const uint32_t *a = g->adj + g->off[u];
        for (uint64_t i = g->row_ptr[u]; i < g->row_ptr[u + 1]; ++i) {
            uint64_t v = a[i - g->row_ptr[u]];
            if (col_bytes == 4) ((uint32_t *)col)[i] = (uint32_t)v;
            else ((uint64_t *)col)[i] = v;
            if (weights) {
                uint64_t lo = u < v ? u : v, hi = u < v ? v : u;
                weights[i] = 1u + (uint32_t)(mix64(wkey ^ ((lo << 32) | hi)) % 255u);
            }
        }
    }
    return 0;
}

/* Renumbers the graph's vertices by new_id[old] (a bijection) in place of the
 * handle: used for locality orders.  Lists are re-sorted. */
int gg_relabel(void *h, const uint64_t *new_id)
{
    gg_graph *g = (gg_graph *)h;
    uint64_t V = g->V;
    uint64_t *rp = (uint64_t *)malloc((V + 1) * sizeof(uint64_t));
    uint32_t *adj = (uint32_t *)malloc((g->E ? g->E : 1) * sizeof(uint32_t));
    if (!rp || !adj) { free(rp); free(adj); return -2; }
    rp[0] = 0;
    uint64_t *deg = (uint64_t *)calloc(V + 1, sizeof(uint64_t));
    if (!deg) { free(rp); free(adj); return -2; }
    for (uint64_t u = 0; u < V; ++u) deg[new_id[u]] = g->row_ptr[u + 1] - g->row_ptr[u];
    for (uint64_t v = 0; v < V; ++v) rp[v + 1] = rp[v] + deg[v];
#pragma omp parallel for schedule(dynamic, 4096)
    for (uint64_t u = 0; u < V; ++u) {
        uint64_t nu = new_id[u], base = rp[nu];
        uint64_t n = g->row_ptr[u + 1] - g->row_ptr[u];
        for (uint64_t j = 0; j < n; ++j) adj[base + j] = (uint32_t)new_id[g->adj[g->off[u] + j]];
        sort_u32(adj + base, n);
    }
    free(deg);
    free(g->row_ptr);
    free(g->adj);
    g->row_ptr = rp;
    g->adj = adj;
    memcpy(g->off, rp, V * sizeof(uint64_t));
    return 0;
}

/* Locality order for the power-law stand-in of crawled graphs: ids are given
 * in first-visit order of a queue walk from the highest-degree vertex
 * (unreached vertices follow in id order), then runs of `run` consecutive new
 * ids are permuted by a seeded Fisher-Yates shuffle (order inside a run kept).
 * Writes new_id[old] (a bijection). */
int gg_locality_order(void *h, uint64_t run, uint64_t seed, uint64_t *new_id)
{
    gg_graph *g = (gg_graph *)h;
    const uint64_t V = g->V;
    uint64_t *order = (uint64_t *)malloc((V ? V : 1) * sizeof(uint64_t));
    unsigned char *seen = (unsigned char *)calloc(V ? V : 1, 1);
    if (!order || !seen || run == 0) { free(order); free(seen); return -2; }
    uint64_t root = 0, best = 0, tail = 0, head = 0;
    for (uint64_t v = 0; v < V; ++v)
        if (g->row_ptr[v + 1] - g->row_ptr[v] > best) { best = g->row_ptr[v + 1] - g->row_ptr[v]; root = v; }
    for (uint64_t start = 0; start <= V; ++start) {
        uint64_t s = start == 0 ? root : start - 1;
        if (V == 0 || seen[s]) continue;
        seen[s] = 1;
        order[tail++] = s;
        while (head < tail) {
            uint64_t u = order[head++];
            const uint32_t *a = g->adj + g->off[u];
            for (uint64_t i = 0; i < g->row_ptr[u + 1] - g->row_ptr[u]; ++i)
                if (!seen[a[i]]) { seen[a[i]] = 1; order[tail++] = a[i]; }
        }
    }
    free(seen);
    /* shuffle whole runs: new position of run r is runperm[r] */
    const uint64_t nruns = (V + run - 1) / run;
    uint64_t *runperm = (uint64_t *)malloc((nruns ? nruns : 1) * sizeof(uint64_t));
    if (!runperm) { free(order); return -2; }
    for (uint64_t r = 0; r < nruns; ++r) runperm[r] = r;
    const uint64_t key = gg_stream_key(seed, 4);
    for (uint64_t r = nruns; r > 1; --r) {
        uint64_t j = draw(key, r) % r, t = runperm[r - 1];
        runperm[r - 1] = runperm[j];
        runperm[j] = t;
    }
    /* the last run may be short: lay runs out in permuted order */
    uint64_t *start = (uint64_t *)malloc((nruns + 1) * sizeof(uint64_t));
    if (!start) { free(order); free(runperm); return -2; }
    uint64_t pos = 0;
    for (uint64_t k = 0; k < nruns; ++k) {
        uint64_t r = runperm[k];
        start[r] = pos;
        pos += (r + 1) * run <= V ? run : V - r * run;
    }
    for (uint64_t i = 0; i < V; ++i) new_id[order[i]] = start[i / run] + i % run;
    free(start);
    free(runperm);
    free(order);
    return 0;
}

void gg_free(void *h)
{
    gg_graph *g = (gg_graph *)h;
    if (!g) return;
    free(g->row_ptr);
    free(g->off);
    free(g->adj);
    free(g);
}
