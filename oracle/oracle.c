/*
 * Oracle: plain, slow, obviously correct CPU definitions of what the
 * zero-copy traversal computes.  TEST INFRASTRUCTURE ONLY: nothing in the
 * product path may link, load or call this file.  It shares no code, header
 * or constant with the HIP library.
 *
 * The paper (EMOGI, Sec. 2.1 and Algorithm 1) only changes HOW the CSR edge
 * list is fetched (Sec. 3.3, Sec. 4.3: merged and aligned reads of zero-copy
 * memory), never WHAT is computed.  So every traversal result below is the
 * textbook definition written out:
 *   - BFS level  : fewest edges on a directed path from the source (Sec. 2.1,
 *                  Algorithm 1 with the "not yet visited" condition).
 *   - SSSP dist  : least total integer weight over directed paths
 *                  (Sec. 5.1 systems compared; Sec. 5.2 integer weights).
 *   - CC label   : smallest vertex id in the vertex's connected component of
 *                  the undirected graph (Sec. 5.4: CC on undirected graphs).
 *   - PageRank   : the power iteration in fixed point (see oracle_pagerank).
 * Unreachable is 0xFFFFFFFF for levels and distances.
 *
 * CSR (Sec. 2.1, Fig. 1): row_ptr[V+1] (uint64), col[E] of 4 or 8 bytes,
 * optional per-edge uint32 weights aligned with col.
 *
 * Return codes: 0 ok, -1 invalid argument, -2 out of host memory,
 * -6 a finite distance does not fit in 32 bits.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_INF32 0xFFFFFFFFu
#define ORC_INF64 UINT64_MAX

static uint64_t col_at(const void *col, int col_bytes, uint64_t i)
{
    if (col_bytes == 4)
        return ((const uint32_t *)col)[i];
    return ((const uint64_t *)col)[i];
}

/* ------------------------------------------------------------------ */
/* CSR validation: row_ptr starts at 0 and never decreases, every     */
/* neighbour id is < V.  Optional: lists ascending without duplicates */
/* or self-loops; optional: symmetric (u->v present iff v->u).        */
/* Returns 0 when valid, else the number of the first failed check.   */
/* ------------------------------------------------------------------ */
static int has_edge_sorted(const uint64_t *row_ptr, const void *col, int cb,
                           uint64_t u, uint64_t v)
{
    uint64_t lo = row_ptr[u], hi = row_ptr[u + 1];
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        uint64_t x = col_at(col, cb, mid);
        if (x == v) return 1;
        if (x < v) lo = mid + 1; else hi = mid;
    }
    return 0;
}

int oracle_validate_csr(uint64_t V, const uint64_t *row_ptr, const void *col,
                        int col_bytes, int want_simple, int want_symmetric)
{
    if (col_bytes != 4 && col_bytes != 8) return -1;
    if (row_ptr[0] != 0) return 1;
    for (uint64_t u = 0; u < V; ++u)
        if (row_ptr[u + 1] < row_ptr[u]) return 2;
    for (uint64_t u = 0; u < V; ++u)
        for (uint64_t i = row_ptr[u]; i < row_ptr[u + 1]; ++i)
            if (col_at(col, col_bytes, i) >= V) return 3;
    if (want_simple || want_symmetric) {
        for (uint64_t u = 0; u < V; ++u)
            for (uint64_t i = row_ptr[u]; i < row_ptr[u + 1]; ++i) {
                uint64_t v = col_at(col, col_bytes, i);
                if (v == u) return 4;
                if (i > row_ptr[u] && col_at(col, col_bytes, i - 1) >= v) return 5;
            }
    }
    if (want_symmetric) {
        for (uint64_t u = 0; u < V; ++u)
            for (uint64_t i = row_ptr[u]; i < row_ptr[u + 1]; ++i) {
                uint64_t v = col_at(col, col_bytes, i);
                if (!has_edge_sorted(row_ptr, col, col_bytes, v, u)) return 6;
            }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* BFS by a FIFO queue (Sec. 2.1, Algorithm 1: the source starts      */
/* active; an unvisited neighbour becomes active one level later).    */
/* ------------------------------------------------------------------ */
int oracle_bfs(uint64_t V, const uint64_t *row_ptr, const void *col,
               int col_bytes, uint64_t src, uint32_t *level)
{
    if (src >= V) return -1;
    uint64_t *queue = (uint64_t *)malloc((V ? V : 1) * sizeof(uint64_t));
    if (!queue) return -2;
    for (uint64_t v = 0; v < V; ++v) level[v] = ORC_INF32;
    uint64_t head = 0, tail = 0;
    level[src] = 0;
    queue[tail++] = src;
    while (head < tail) {
        uint64_t u = queue[head++];
        for (uint64_t i = row_ptr[u]; i < row_ptr[u + 1]; ++i) {
            uint64_t v = col_at(col, col_bytes, i);
            if (level[v] == ORC_INF32) {
                level[v] = level[u] + 1;
                queue[tail++] = v;
            }
        }
    }
    free(queue);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Dijkstra with a binary min-heap of (distance, vertex) and lazy      */
/* deletion.  Distances are kept in 64 bits; at the end a finite value */
/* above 0xFFFFFFFE is reported as an overflow (-6).                   */
/* ------------------------------------------------------------------ */
typedef struct { uint64_t d, v; } heap_item;

static void heap_push(heap_item *h, uint64_t *n, heap_item x)
{
    uint64_t i = (*n)++;
    h[i] = x;
    while (i > 0) {
        uint64_t p = (i - 1) / 2;
        if (h[p].d <= h[i].d) break;
        heap_item t = h[p]; h[p] = h[i]; h[i] = t;
        i = p;
    }
}

static heap_item heap_pop(heap_item *h, uint64_t *n)
{
    heap_item top = h[0];
    h[0] = h[--(*n)];
    uint64_t i = 0;
    for (;;) {
        uint64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < *n && h[l].d < h[m].d) m = l;
        if (r < *n && h[r].d < h[m].d) m = r;
        if (m == i) break;
        heap_item t = h[m]; h[m] = h[i]; h[i] = t;
        i = m;
    }
    return top;
}

int oracle_dijkstra(uint64_t V, const uint64_t *row_ptr, const void *col,
                    int col_bytes, const uint32_t *w, uint64_t src,
                    uint32_t *dist)
{
    if (src >= V || !w) return -1;
    uint64_t E = row_ptr[V];
    uint64_t *d = (uint64_t *)malloc((V ? V : 1) * sizeof(uint64_t));
    /* every successful relaxation pushes once, plus the source */
    heap_item *h = (heap_item *)malloc((E + 1) * sizeof(heap_item));
    if (!d || !h) { free(d); free(h); return -2; }
    for (uint64_t v = 0; v < V; ++v) d[v] = ORC_INF64;
    uint64_t n = 0;
    d[src] = 0;
    heap_item s = {0, src};
    heap_push(h, &n, s);
    while (n > 0) {
        heap_item top = heap_pop(h, &n);
        uint64_t u = top.v;
        if (top.d > d[u]) continue; /* stale entry */
        for (uint64_t i = row_ptr[u]; i < row_ptr[u + 1]; ++i) {
            uint64_t v = col_at(col, col_bytes, i);
            uint64_t nd = top.d + (uint64_t)w[i];
            if (nd < d[v]) {
                d[v] = nd;
                heap_item x = {nd, v};
                heap_push(h, &n, x);
            }
        }
    }
    int rc = 0;
    for (uint64_t v = 0; v < V; ++v) {
        if (d[v] == ORC_INF64) dist[v] = ORC_INF32;
        else if (d[v] > 0xFFFFFFFEull) { dist[v] = ORC_INF32; rc = -6; }
        else dist[v] = (uint32_t)d[v];
    }
    free(d);
    free(h);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Connected components by union-find.  Union always hangs the larger */
/* root below the smaller one, so every root is its set's minimum id; */
/* the label of v is then the root of v.  Edges are taken undirected.  */
/* ------------------------------------------------------------------ */
static uint64_t uf_find(uint64_t *parent, uint64_t x)
{
    while (parent[x] != x) {
        parent[x] = parent[parent[x]]; /* path halving */
        x = parent[x];
    }
    return x;
}

int oracle_cc(uint64_t V, const uint64_t *row_ptr, const void *col,
              int col_bytes, uint32_t *label)
{
    uint64_t *parent = (uint64_t *)malloc((V ? V : 1) * sizeof(uint64_t));
    if (!parent) return -2;
    for (uint64_t v = 0; v < V; ++v) parent[v] = v;
    for (uint64_t u = 0; u < V; ++u)
        for (uint64_t i = row_ptr[u]; i < row_ptr[u + 1]; ++i) {
            uint64_t a = uf_find(parent, u);
            uint64_t b = uf_find(parent, col_at(col, col_bytes, i));
            if (a < b) parent[b] = a;
            else if (b < a) parent[a] = b;
        }
    for (uint64_t v = 0; v < V; ++v) label[v] = (uint32_t)uf_find(parent, v);
    free(parent);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Floyd-Warshall all-pairs distances on a tiny graph (n <= a few     */
/* hundred).  w == NULL means every edge weighs 1 (BFS levels).       */
/* D is n*n uint64, row = source; unreachable = UINT64_MAX.           */
/* ------------------------------------------------------------------ */
int oracle_floyd_warshall(uint64_t n, const uint64_t *row_ptr, const void *col,
                          int col_bytes, const uint32_t *w, uint64_t *D)
{
    for (uint64_t i = 0; i < n * n; ++i) D[i] = ORC_INF64;
    for (uint64_t i = 0; i < n; ++i) D[i * n + i] = 0;
    for (uint64_t u = 0; u < n; ++u)
        for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            uint64_t v = col_at(col, col_bytes, e);
            uint64_t c = w ? (uint64_t)w[e] : 1;
            if (c < D[u * n + v]) D[u * n + v] = c;
        }
    for (uint64_t k = 0; k < n; ++k)
        for (uint64_t i = 0; i < n; ++i) {
            if (D[i * n + k] == ORC_INF64) continue;
            for (uint64_t j = 0; j < n; ++j) {
                if (D[k * n + j] == ORC_INF64) continue;
                uint64_t c = D[i * n + k] + D[k * n + j];
                if (c < D[i * n + j]) D[i * n + j] = c;
            }
        }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Brute-force CC on a tiny graph: boolean transitive closure of the  */
/* undirected adjacency (Warshall), then label = least reachable id.  */
/* ------------------------------------------------------------------ */
int oracle_cc_closure(uint64_t n, const uint64_t *row_ptr, const void *col,
                      int col_bytes, uint32_t *label)
{
    unsigned char *R = (unsigned char *)calloc((n > 0) ? n * n : 1, 1);
    if (!R) return -2;
    for (uint64_t i = 0; i < n; ++i) R[i * n + i] = 1;
    for (uint64_t u = 0; u < n; ++u)
        for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            uint64_t v = col_at(col, col_bytes, e);
            R[u * n + v] = 1;
            R[v * n + u] = 1;
        }
    for (uint64_t k = 0; k < n; ++k)
        for (uint64_t i = 0; i < n; ++i)
            if (R[i * n + k])
                for (uint64_t j = 0; j < n; ++j)
                    if (R[k * n + j]) R[i * n + j] = 1;
    for (uint64_t v = 0; v < n; ++v) {
        uint64_t m = v;
        for (uint64_t u = 0; u < n; ++u)
            if (R[v * n + u] && u < m) m = u;
        label[v] = (uint32_t)m;
    }
    free(R);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Linear-time certificate for a distance vector d from src with all  */
/* weights >= 1 (w == NULL: unit weights, i.e. BFS levels):           */
/*   1. d[src] == 0                                                    */
/*   2. every edge u->v with d[u] finite has d[v] <= d[u] + w          */
/*   3. every v != src with d[v] finite has an in-edge u->v, d[u]      */
/*      finite, with d[u] + w == d[v]                                   */
/* Together they hold iff d is exactly the distance vector.            */
/* Returns 0 when certified, else the number of the failed condition.  */
/* ------------------------------------------------------------------ */
int oracle_certify_distances(uint64_t V, const uint64_t *row_ptr,
                             const void *col, int col_bytes,
                             const uint32_t *w, uint64_t src,
                             const uint32_t *d)
{
    if (src >= V) return -1;
    if (d[src] != 0) return 1;
    unsigned char *tight = (unsigned char *)calloc(V ? V : 1, 1);
    if (!tight) return -2;
    int rc = 0;
    /* The loops are independent per vertex; they run on all cores so the
     * check stays affordable on billions of edges.  Failure codes combine
     * with max (-1 < 2 < 3 never mix: each is reported alone below). */
    int bad_weight = 0, bad_edge = 0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(| : bad_weight, bad_edge)
    for (uint64_t u = 0; u < V; ++u) {
        if (d[u] == ORC_INF32) continue;
        for (uint64_t i = row_ptr[u]; i < row_ptr[u + 1]; ++i) {
            uint64_t v = col_at(col, col_bytes, i);
            uint64_t c = w ? (uint64_t)w[i] : 1;
            if (c == 0) { bad_weight = 1; break; }
            uint64_t nd = (uint64_t)d[u] + c;
            uint64_t dv = d[v] == ORC_INF32 ? ORC_INF64 : (uint64_t)d[v];
            if (dv > nd) { bad_edge = 1; break; }
            if (dv == nd) __atomic_store_n(&tight[v], 1, __ATOMIC_RELAXED);
        }
    }
    if (bad_weight) rc = -1;
    else if (bad_edge) rc = 2;
    if (!rc) {
        int untight = 0;
#pragma omp parallel for reduction(| : untight)
        for (uint64_t v = 0; v < V; ++v)
            if (v != src && d[v] != ORC_INF32 && !tight[v]) untight = 1;
        if (untight) rc = 3;
    }
    free(tight);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Certificate for CC labels on a symmetric graph:                     */
/*   1. label equal across every edge                                  */
/*   2. label[v] <= v and label[label[v]] == label[v]                  */
/*   3. number of distinct labels == number of union-find components   */
/* Returns 0 when certified, else the failed condition.                */
/* ------------------------------------------------------------------ */
int oracle_certify_cc(uint64_t V, const uint64_t *row_ptr, const void *col,
                      int col_bytes, const uint32_t *label)
{
    for (uint64_t u = 0; u < V; ++u)
        for (uint64_t i = row_ptr[u]; i < row_ptr[u + 1]; ++i)
            if (label[u] != label[col_at(col, col_bytes, i)]) return 1;
    uint64_t roots = 0;
    for (uint64_t v = 0; v < V; ++v) {
        if ((uint64_t)label[v] > v) return 2;
        if (label[label[v]] != label[v]) return 2;
        if (label[v] == v) ++roots;
    }
    uint32_t *uf = (uint32_t *)malloc((V ? V : 1) * sizeof(uint32_t));
    if (!uf) return -2;
    int rc = oracle_cc(V, row_ptr, col, col_bytes, uf);
    if (rc == 0) {
        uint64_t comps = 0;
        for (uint64_t v = 0; v < V; ++v) if (uf[v] == v) ++comps;
        if (comps != roots) rc = 3;
    }
    free(uf);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Host-link bytes a request-granular scan of neighbour lists moves    */
/* (Sec. 3.3 request sizes; Sec. 4.3.2 aligned access): a list that    */
/* occupies bytes [e*s, e*t) of the edge array costs every R-byte      */
/* block it overlaps.  mask[v] != 0 selects the scanned vertices       */
/* (mask == NULL: all).  Empty lists cost nothing.                     */
/* ------------------------------------------------------------------ */
uint64_t oracle_request_bytes(uint64_t V, const uint64_t *row_ptr,
                              int elem_bytes, uint64_t R,
                              const unsigned char *mask)
{
    uint64_t total = 0;
    for (uint64_t v = 0; v < V; ++v) {
        if (mask && !mask[v]) continue;
        uint64_t s = row_ptr[v], t = row_ptr[v + 1];
        if (t == s) continue;
        uint64_t first = (s * (uint64_t)elem_bytes) / R;
        uint64_t last = (t * (uint64_t)elem_bytes + R - 1) / R;
        total += (last - first) * R;
    }
    return total;
}

/* Sum of out-degrees over the vertices whose distance is finite: the  */
/* edges a traversal from the source must read (TEPS numerator).       */
uint64_t oracle_reached_edges(uint64_t V, const uint64_t *row_ptr,
                              const uint32_t *d)
{
    uint64_t total = 0;
    for (uint64_t v = 0; v < V; ++v)
        if (d[v] != ORC_INF32) total += row_ptr[v + 1] - row_ptr[v];
    return total;
}

/* ------------------------------------------------------------------ */
/* PageRank (EMOGI's fourth workload, Sec. 5.1 and Sec. 5.4), pull     */
/* form on an undirected graph, in fixed point so that every sum is   */
/* exact and the result cannot depend on the order of additions.      */
/* With one = 2^F and d the damping factor scaled to an integer        */
/* (d < one):                                                          */
/*   pr_0(v)     = floor(one / V)                                     */
/*   c_t(u)      = floor(pr_t(u) / deg(u))   (0 when deg(u) = 0)       */
/*   s_t(v)      = sum of c_t(u) over the neighbours u of v            */
/*   pr_{t+1}(v) = floor((one - d) / V) + floor(d * s_t(v) / one)      */
/* A vertex without neighbours passes no score on (no redistribution). */
/* Scores stay below one, so d * s fits in 128 bits.                   */
/* ------------------------------------------------------------------ */
int oracle_pagerank(uint64_t V, const uint64_t *row_ptr, const void *col,
                    int col_bytes, uint32_t frac_bits, uint64_t d,
                    uint32_t iters, uint64_t *pr)
{
    if (frac_bits < 1 || frac_bits > 62) return -1;
    const uint64_t one = (uint64_t)1 << frac_bits;
    if (d >= one) return -1;
    if (V == 0) return 0;
    uint64_t *c = (uint64_t *)malloc(V * sizeof(uint64_t));
    if (!c) return -2;
    const uint64_t base = (one - d) / V;
    for (uint64_t v = 0; v < V; ++v) pr[v] = one / V;
    for (uint32_t t = 0; t < iters; ++t) {
        for (uint64_t u = 0; u < V; ++u) {
            uint64_t deg = row_ptr[u + 1] - row_ptr[u];
            c[u] = deg ? pr[u] / deg : 0;
        }
        for (uint64_t v = 0; v < V; ++v) {
            uint64_t s = 0;
            for (uint64_t i = row_ptr[v]; i < row_ptr[v + 1]; ++i)
                s += c[col_at(col, col_bytes, i)];
            unsigned __int128 prod = (unsigned __int128)d * s;
            pr[v] = base + (uint64_t)(prod >> frac_bits);
        }
    }
    free(c);
    return 0;
}
