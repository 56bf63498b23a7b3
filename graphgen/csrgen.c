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
 *     distribution by inversion of the prefix table.
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
    const double *cdf;      /* Chung-Lu: cumulative weights, length V */
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
            int rb, cb;
            if (r < s->ta) { rb = 0; cb = 0; }
            else if (r < s->tab) { rb = 0; cb = 1; }
            else if (r < s->tabc) { rb = 1; cb = 0; }
            else { rb = 1; cb = 1; }
            u = (u << 1) | (uint64_t)rb;
            v = (v << 1) | (uint64_t)cb;
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
        /* inversion: first index whose cumulative weight exceeds r */
        for (int e = 0; e < 2; ++e) {
            double r = (double)(draw(s->key, 2 * k + (uint64_t)e) >> 11) * (1.0 / 9007199254740992.0);
            r *= s->cdf[s->V - 1];
            uint64_t lo = 0, hi = s->V - 1;
            while (lo < hi) {
                uint64_t mid = lo + (hi - lo) / 2;
                if (s->cdf[mid] > r) hi = mid; else lo = mid + 1;
            }
            if (e == 0) u = lo; else v = lo;
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

static void sort_u32(uint32_t *a, uint64_t n)
{
    if (n < 32) { /* insertion sort for short lists */
        for (uint64_t i = 1; i < n; ++i) {
            uint32_t x = a[i];
            uint64_t j = i;
            while (j > 0 && a[j - 1] > x) { a[j] = a[j - 1]; --j; }
            a[j] = x;
        }
    } else {
        qsort(a, n, sizeof(uint32_t), cmp_u32);
    }
}

/* Builds the simple symmetric graph of the sampler's m samples. */
static gg_graph *build(const sampler_t *s)
{
    uint64_t V = s->V, m = s->m;
    gg_graph *g = (gg_graph *)calloc(1, sizeof(gg_graph));
    uint32_t *deg = (uint32_t *)calloc(V, sizeof(uint32_t));
    uint64_t *off = (uint64_t *)malloc((V + 1) * sizeof(uint64_t));
    uint64_t *pos = (uint64_t *)malloc(V * sizeof(uint64_t));
    if (!g || !deg || !off || !pos) goto fail;

#pragma omp parallel for schedule(static, 65536)
    for (uint64_t k = 0; k < m; ++k) {
        uint64_t u, v;
        sample_edge(s, k, &u, &v);
        if (u == v) continue;
        __atomic_fetch_add(&deg[u], 1u, __ATOMIC_RELAXED);
        __atomic_fetch_add(&deg[v], 1u, __ATOMIC_RELAXED);
    }
    off[0] = 0;
    for (uint64_t v = 0; v < V; ++v) off[v + 1] = off[v] + deg[v];
    uint64_t total = off[V];
    g->adj = (uint32_t *)malloc((total ? total : 1) * sizeof(uint32_t));
    if (!g->adj) goto fail;
    memcpy(pos, off, V * sizeof(uint64_t));

#pragma omp parallel for schedule(static, 65536)
    for (uint64_t k = 0; k < m; ++k) {
        uint64_t u, v;
        sample_edge(s, k, &u, &v);
        if (u == v) continue;
        uint64_t pu = __atomic_fetch_add(&pos[u], 1ull, __ATOMIC_RELAXED);
        uint64_t pv = __atomic_fetch_add(&pos[v], 1ull, __ATOMIC_RELAXED);
        g->adj[pu] = (uint32_t)v;
        g->adj[pv] = (uint32_t)u;
    }
    free(pos);
    pos = NULL;

    /* sort + unique each list in place; deg[v] becomes the unique count */
#pragma omp parallel for schedule(dynamic, 4096)
    for (uint64_t v = 0; v < V; ++v) {
        uint32_t *a = g->adj + off[v];
        uint64_t n = off[v + 1] - off[v];
        sort_u32(a, n);
        uint64_t w = 0;
        for (uint64_t i = 0; i < n; ++i)
            if (i == 0 || a[i] != a[w - 1]) a[w++] = a[i];
        deg[v] = (uint32_t)w;
    }
    g->row_ptr = (uint64_t *)malloc((V + 1) * sizeof(uint64_t));
    if (!g->row_ptr) goto fail;
    g->row_ptr[0] = 0;
    for (uint64_t v = 0; v < V; ++v) g->row_ptr[v + 1] = g->row_ptr[v] + deg[v];
    g->E = g->row_ptr[V];
    g->V = V;
    g->off = off;
    free(deg);
    return g;
fail:
    if (g) { free(g->adj); free(g->row_ptr); free(g); }
    free(deg); free(off); free(pos);
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
    double *cdf = (double *)malloc(V * sizeof(double));
    if (!cdf) return NULL;
    double acc = 0.0, expo = -1.0 / (gamma - 1.0);
    for (uint64_t i = 0; i < V; ++i) {
        acc += pow((double)i + i0, expo);
        cdf[i] = acc;
    }
    s.kind = GG_CHUNGLU;
    s.V = V;
    s.m = samples;
    s.key = gg_stream_key(seed, STREAM_EDGES);
    s.cdf = cdf;
    s.permute = permute;
    perm_init(&s.perm, seed, V);
    gg_graph *g = build(&s);
    free(cdf);
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

void gg_free(void *h)
{
    gg_graph *g = (gg_graph *)h;
    if (!g) return;
    free(g->row_ptr);
    free(g->off);
    free(g->adj);
    free(g);
}
