/*
 * emogi.h - C ABI of the MI355X zero-copy graph traversal library.
 *
 * The library traverses a CSR graph (EMOGI Sec. 2.1, Fig. 1: a vertex list
 * of offsets and an edge list of neighbour ids) whose edge list may stay in
 * pinned host memory and be read in place by the GPU over the host link
 * (Sec. 3.1 enabling zero-copy; Sec. 4.2: edge list in host memory, vertex
 * list and per-vertex buffers in GPU memory, all mapped once at set-up).
 * Neighbour lists are scanned by wave-wide merged reads whose start is
 * rounded down to the link's request unit (Sec. 4.3.1 merged access,
 * Sec. 4.3.2 aligned access), one frontier level per step (Sec. 4.2,
 * Algorithm 1).
 *
 * Conventions shared by every call
 *   - Status codes are returned, never thrown; emogi_last_error() gives a
 *     thread-local message for the last failing call on this thread.
 *   - Host inputs are plain host pointers; they are copied at create time
 *     unless EMOGI_F_BORROW is given.
 *   - Outputs (levels, dist, labels) are device pointers (hipMalloc'd memory,
 *     e.g. a torch HIP tensor's data_ptr) of at least V (or n*V) uint32.
 *   - `stream` is a hipStream_t passed as void* (NULL: the null stream).
 *     Traversal calls enqueue on it and return after the traversal has
 *     finished: each level needs the next frontier's length on the host.
 *   - One traversal at a time per graph handle (it owns the scratch pool).
 *   - Unreachable vertices get 0xFFFFFFFF (EMOGI_INF).
 */
#ifndef EMOGI_H
#define EMOGI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EMOGI_INF 0xFFFFFFFFu

typedef struct emogi_graph_s *emogi_graph_t; /* opaque, library-owned */

typedef enum {
    EMOGI_PLACE_HBM = 0,            /* edge list copied into GPU memory              */
    EMOGI_PLACE_HOST_ZERO_COPY = 1, /* edge list in pinned host memory, read in place */
    EMOGI_PLACE_MANAGED = 2         /* edge list in hipMallocManaged memory (UVM arm, Sec. 5.1 (a)) */
} emogi_placement_t;

typedef enum {
    EMOGI_OK = 0,
    EMOGI_E_INVALID = -1,       /* bad argument or malformed CSR                 */
    EMOGI_E_OOM_HOST = -2,      /* host or pinned allocation failed              */
    EMOGI_E_OOM_DEVICE = -3,    /* device allocation failed                      */
    EMOGI_E_HIP = -4,           /* a HIP runtime call failed                     */
    EMOGI_E_NOT_SYMMETRIC = -5, /* CC needs an undirected (symmetric) graph      */
    EMOGI_E_OVERFLOW = -6,      /* a finite SSSP distance exceeds 0xFFFFFFFE     */
    EMOGI_E_NOCONVERGE = -7,    /* iteration cap reached                         */
    EMOGI_E_UNSUPPORTED = -8    /* placement or size not supported on this GPU   */
} emogi_status_t;

/* emogi_graph_create flags */
#define EMOGI_F_SYMMETRIC 0x1u       /* caller asserts u->v present iff v->u (needed by CC) */
#define EMOGI_F_VALIDATE 0x2u        /* O(V+E) host check of the CSR (and symmetry if flagged) */
#define EMOGI_F_BORROW 0x4u          /* col/weights were allocated by emogi_host_alloc: use them
                                        in place (zero-copy placement only); the caller keeps them
                                        alive and unmodified until emogi_graph_destroy */
#define EMOGI_F_PIN_NONCOHERENT 0x8u /* pinned edge list allocated non-coherent */

/* Access variants of the neighbour scan (all give identical results). */
typedef enum {
    EMOGI_V0_THREAD = 0,     /* one thread per vertex, element by element (Sec. 4.2, naive)   */
    EMOGI_V1_GROUP16 = 1,    /* 16-lane group per vertex, start aligned                      */
    EMOGI_V2_WAVE = 2,       /* wave64 per vertex, merged, unaligned (Sec. 4.3.1)             */
    EMOGI_V3_WAVE_ALIGNED = 3, /* wave64 per vertex, merged + aligned (Sec. 4.3.2)           */
    EMOGI_V4_BLOCK = 4,      /* 256-thread workgroup per vertex, aligned                      */
    EMOGI_V5_BALANCED = 5,   /* aligned chunks of all frontier lists dealt out evenly to waves */
    EMOGI_NUM_VARIANTS = 6
} emogi_variant_t;

/* Scheduler modes for emogi_set_scheduler. */
#define EMOGI_SCHED_FIXED(v) ((int)(v)) /* always variant v (0..5)                   */
#define EMOGI_SCHED_HEURISTIC 16        /* rule of thumb on frontier size and degrees */
#define EMOGI_SCHED_LEARNED 17          /* MLP over frontier features (falls back to the
                                           heuristic when no weights are loaded)       */

#define EMOGI_MAX_LEVEL_STATS 512

typedef struct {
    uint32_t iterations;         /* levels (BFS) or rounds (SSSP, CC) executed           */
    uint32_t variant_hist[EMOGI_NUM_VARIANTS]; /* how many levels each variant ran     */
    uint64_t vertices_expanded;  /* frontier entries whose lists were scanned            */
    uint64_t edges_scanned;      /* sum of their out-degrees (re-expansions included)    */
    uint64_t useful_link_bytes;  /* edges_scanned * (col_bytes + 4 if weights read)      */
    uint64_t request_bytes;      /* the same lists rounded out to the request unit R     */
    double total_ms;             /* whole traversal, HIP events on the caller's stream   */
    double expand_ms;            /* sum of the neighbour-scan kernels alone              */
    uint32_t expand_launches;    /* how many neighbour-scan kernels ran                  */
    uint32_t request_unit;       /* R in bytes used for alignment                        */
    uint32_t level_count;        /* entries filled in the per-level arrays below         */
    uint8_t level_variant[EMOGI_MAX_LEVEL_STATS];
    uint32_t level_frontier[EMOGI_MAX_LEVEL_STATS];
    float level_ms[EMOGI_MAX_LEVEL_STATS];   /* neighbour-scan kernel time per level     */
    uint64_t level_edges[EMOGI_MAX_LEVEL_STATS]; /* edges scanned per level               */
} emogi_stats_t;

/* ---- pinned host memory for EMOGI_F_BORROW (Sec. 3.1: the edge list must be
 *      pinned and mapped into the GPU's address space) ---- */
/* Allocates `bytes` of pinned, GPU-mapped host memory.  *out receives a host
 * pointer that the GPU can also dereference.  EMOGI_E_OOM_HOST on failure. */
emogi_status_t emogi_host_alloc(size_t bytes, uint32_t flags, void **out);
emogi_status_t emogi_host_free(void *p);

/* ---- graph handle (Sec. 4.2: everything is mapped once at set-up) ----
 * row_ptr     host uint64[num_vertices+1], row_ptr[0] == 0, non-decreasing;
 *             E = row_ptr[V].  Copied into GPU memory.
 * col         host array of E neighbour ids, col_bytes = 4 or 8, each < V.
 * weights     host uint32[E] edge weights (NULL: SSSP unavailable).
 * placement   where col and weights live (see emogi_placement_t).
 * Errors: EMOGI_E_INVALID (bad sizes, V >= 2^32-1, malformed CSR under
 * EMOGI_F_VALIDATE, BORROW of memory not from emogi_host_alloc),
 * EMOGI_E_NOT_SYMMETRIC (EMOGI_F_VALIDATE|EMOGI_F_SYMMETRIC on an asymmetric
 * graph), EMOGI_E_OOM_*, EMOGI_E_UNSUPPORTED (placement not available).
 * Nothing is leaked on failure; *out is set only on success. */
emogi_status_t emogi_graph_create(const uint64_t *row_ptr, uint64_t num_vertices,
                                  const void *col, uint32_t col_bytes,
                                  const uint32_t *weights, emogi_placement_t placement,
                                  uint32_t flags, emogi_graph_t *out);
emogi_status_t emogi_graph_destroy(emogi_graph_t g);

/* Request unit R (bytes, power of two 32..4096) used to round list starts
 * down (Sec. 4.3.2).  Default 256: the smallest block that runs the MI355X
 * host link at its copy rate when read at random. */
emogi_status_t emogi_set_request_unit(emogi_graph_t g, uint32_t bytes);
emogi_status_t emogi_set_scheduler(emogi_graph_t g, int mode);
/* Loads the 5638 fp32 scheduler parameters (order W1,b1,W2,b2,W3,b3, row-major)
 * from host memory; NULL clears them (learned mode then uses the heuristic). */
emogi_status_t emogi_set_scheduler_weights(emogi_graph_t g, const float *params, size_t count);

/* ---- traversals (Sec. 5.1: BFS, SSSP, CC) ----
 * emogi_bfs : levels[v] = fewest edges on a path src->v (src gets 0).
 * emogi_sssp: dist[v] = least sum of weights over paths src->v; needs weights;
 *             EMOGI_E_OVERFLOW if a reachable vertex's distance exceeds
 *             0xFFFFFFFE (dist contents are then unspecified).
 * emogi_cc  : labels[v] = smallest vertex id in v's connected component; needs
 *             a graph created with EMOGI_F_SYMMETRIC (else EMOGI_E_NOT_SYMMETRIC).
 * src >= V gives EMOGI_E_INVALID. */
emogi_status_t emogi_bfs(emogi_graph_t g, uint64_t src, uint32_t *levels, void *stream);
emogi_status_t emogi_sssp(emogi_graph_t g, uint64_t src, uint32_t *dist, void *stream);
emogi_status_t emogi_cc(emogi_graph_t g, uint32_t *labels, void *stream);

/* Statistics of the last traversal on this handle. */
emogi_status_t emogi_last_stats(emogi_graph_t g, emogi_stats_t *out);

/* Graph facts. */
uint64_t emogi_num_vertices(emogi_graph_t g);
uint64_t emogi_num_edges(emogi_graph_t g);

const char *emogi_strerror(emogi_status_t e);
const char *emogi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EMOGI_H */
