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
#define EMOGI_F_PACK 0x10u           /* store the lists compressed (see emogi_packed_bytes) */
#define EMOGI_F_WEIGHT_BOUND 0x20u   /* compute weight bounds at creation (see emogi_graph_create) */

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
#define EMOGI_SCHED_LEARNED 17          /* MLP over frontier features: argmax over the
                                           variants whose worker fits the frontier's
                                           longest list (a thread below 16 ids, a
                                           16-lane group below 64, a wave below 4096;
                                           V4 and V5 always); the heuristic when no
                                           weights are loaded, a feature lies outside
                                           the trained range, or the frontier is one
                                           vertex                                      */
#define EMOGI_SCHED_PROBE 18            /* time all six variants on every level (state is
                                           saved and restored), then run the fastest: the
                                           per-level best that training labels come from */
#define EMOGI_SCHED_RECORD 0x100        /* OR into any mode: keep each level's 16 features */
#define EMOGI_NUM_FEATURES 16

#define EMOGI_MAX_LEVEL_STATS 512

typedef struct {
    uint32_t iterations;         /* levels (BFS) or rounds (SSSP, CC) executed           */
    uint32_t variant_hist[EMOGI_NUM_VARIANTS]; /* how many levels each variant ran     */
    uint64_t vertices_expanded;  /* frontier entries whose lists were scanned            */
    uint64_t edges_scanned;      /* sum of their out-degrees (re-expansions included)    */
    uint64_t useful_link_bytes;  /* (edges_scanned - tier_edges) * col_bytes
                                    + 4 * weights_read: bytes the lists need from the link
                                    (packed graphs: the encoded bytes of the lists scanned,
                                    and of their weights for SSSP)                          */
    uint64_t request_bytes;      /* the same lists rounded out to the request unit R     */
    uint64_t tier_edges;         /* of edges_scanned, those read from the HBM tier       */
    uint64_t weights_read;       /* SSSP: weights read over the host link (a weight is
                                    read only when its edge could improve the target:
                                    dist(v) > dist(u) + the smallest weight into v,
                                    or into any vertex when the edges are in HBM;
                                    0 on packed graphs, whose weights come packed)    */
    double total_ms;             /* whole traversal, HIP events on the caller's stream   */
    double expand_ms;            /* sum of the neighbour-scan kernels alone              */
    uint32_t expand_launches;    /* how many neighbour-scan kernels ran                  */
    uint32_t request_unit;       /* R in bytes used for alignment                        */
    uint32_t level_count;        /* entries filled in the per-level arrays below         */
    uint8_t level_variant[EMOGI_MAX_LEVEL_STATS];
    uint32_t level_frontier[EMOGI_MAX_LEVEL_STATS];
    float level_ms[EMOGI_MAX_LEVEL_STATS];   /* neighbour-scan kernel time per level     */
    uint64_t level_edges[EMOGI_MAX_LEVEL_STATS]; /* edges scanned per level               */
    /* frontier features per level (EMOGI_SCHED_RECORD): log2(1+|F|)/32, |F|/V,
     * log2(1+sum deg)/40, sum deg/E, fractions of frontier degrees in <=1, [2,4),
     * [4,8), [8,16), [16,64), [64,256), [256,4096), >=4096, 8-byte ids, weights
     * read, zero-copy placement, managed placement */
    float level_features[EMOGI_MAX_LEVEL_STATS][EMOGI_NUM_FEATURES];
    float level_probe_ms[EMOGI_MAX_LEVEL_STATS][EMOGI_NUM_VARIANTS]; /* EMOGI_SCHED_PROBE: each
                                    variant's level time, its preparation kernels included */
    double prep_ms;              /* of expand_ms: the preparation kernels of the levels (the
                                    edge-balanced variant's chunk prefix) and CC's sampling pass */
    uint64_t reached_edges;      /* BFS, SSSP: sum of out-degrees of the reached vertices (the
                                    TEPS numerator); CC, PageRank: all edges                   */
    uint64_t id_sector_bytes;    /* neighbour-id bytes read over the host link at 32-byte sector
                                    granularity (each list, or each bottom-up read, rounded out
                                    to whole sectors)                                          */
    uint64_t weight_sector_bytes;/* SSSP: 32-byte weight sectors holding a weight read over the
                                    host link, x 32 (several weights of one sector count once)  */
    uint32_t levels_by_network;  /* levels whose variant the scheduler network picked          */
    uint32_t bottom_up_levels;   /* BFS levels run bottom-up (emogi_set_direction)             */
    uint8_t level_direction[EMOGI_MAX_LEVEL_STATS]; /* 0 top-down, 1 bottom-up                  */
} emogi_stats_t;

/* ---- host-link calibration (the MI355X counterpart of the paper's toy 1-D
 *      zero-copy copy study, Sec. 3.3 and Fig. 4) ---- */
#define EMOGI_CALIB_BLOCKS 8  /* random-read block sizes 32, 64, ..., 4096 bytes */
#define EMOGI_CALIB_WAVES 10  /* waves in flight 16, 32, ..., 8192 */
#define EMOGI_CALIB_OFFSETS 17 /* block start offsets 0, s, 2s, ..., 16s with s = max(16, R/16) */
typedef struct {
    double memcpy_GBps;        /* hipMemcpy pinned host -> device, best of 3 (Sec. 5.3.2's peak) */
    double seq_read_GBps[3];   /* wave-merged sequential kernel reads, 4/8/16-byte lanes        */
    uint32_t block_bytes[EMOGI_CALIB_BLOCKS];
    double rand_aligned_GBps[EMOGI_CALIB_BLOCKS]; /* random blocks starting on a block boundary  */
    double rand_shift32_GBps[EMOGI_CALIB_BLOCKS]; /* the same blocks shifted by 32 bytes        */
    uint32_t request_unit;     /* R: smallest aligned block reaching 90% of the sequential rate  */
    double latency_us;         /* dependent-load round trip to pinned host memory                */
    uint64_t buffer_bytes;     /* size of the pinned buffer used                                 */
    /* Little's law (Sec. 3.3): random aligned R-byte blocks read by a fixed
     * number of waves, each with one block in flight at a time */
    uint32_t waves[EMOGI_CALIB_WAVES];
    double waves_GBps[EMOGI_CALIB_WAVES];
    uint32_t knee_waves;       /* fewest waves reaching 90% of the sweep's best rate             */
    /* Fig. 4 (b) vs (c): random R-byte blocks whose start lies `offset` bytes
     * past an R boundary (each block then spans two request units unless 0 or R) */
    uint32_t offset_bytes[EMOGI_CALIB_OFFSETS];
    double offset_GBps[EMOGI_CALIB_OFFSETS];
    /* the same buffer size pinned non-coherent (hipHostMallocNonCoherent) */
    double nc_memcpy_GBps;
    double nc_seq_read_GBps;   /* 16-byte lanes */
    double nc_rand_GBps;       /* random aligned R-byte blocks */
    double coh_rand_GBps;      /* the coherent buffer, same kernel and launch as nc_rand_GBps */
    /* GPU memory (HBM) for the vertex state: a wave-merged read of a device
     * buffer, and a device-to-device copy counted as read + write bytes */
    double hbm_read_GBps;
    double hbm_copy_GBps;
} emogi_link_profile_t;

/* Measures the host link with a pinned buffer of `bytes` (>= 64 MiB; a few GiB
 * recommended) on the current device and null stream, and GPU memory with a
 * device buffer of the same size.  Allocates and frees its own memory (two
 * pinned buffers, coherent and non-coherent, and two device buffers).
 * EMOGI_E_OOM_* when the buffers cannot be allocated. */
emogi_status_t emogi_calibrate_link(size_t bytes, emogi_link_profile_t *out);

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
 *             By default creation reads no weight: the lists are mapped and
 *             nothing is preprocessed.  With EMOGI_F_WEIGHT_BOUND it finds
 *             the smallest weight (a host pass) and, in host zero-copy
 *             placement, each vertex's smallest incoming weight (one GPU
 *             pass over col and weights across the link, V bytes of GPU
 *             memory; its time is reported by emogi_graph_setup_ms); SSSP
 *             then skips the weight read of every edge that cannot improve
 *             its target (dist(v) <= dist(u) + that bound).  Without the
 *             bounds it skips those with dist(v) <= dist(u).
 * placement   where col and weights live (see emogi_placement_t).
 * Errors: EMOGI_E_INVALID (bad sizes, V >= 2^32-1, malformed CSR under
 * EMOGI_F_VALIDATE, BORROW of memory not from emogi_host_alloc),
 * EMOGI_E_NOT_SYMMETRIC (EMOGI_F_VALIDATE|EMOGI_F_SYMMETRIC on an asymmetric
 * graph), EMOGI_E_OOM_*, EMOGI_E_UNSUPPORTED (placement not available).
 * EMOGI_F_PACK stores the lists compressed, the data compression with
 * decoding on the GPU that Sec. 6 proposes to cut link traffic: each list
 * (ascending ids required, else EMOGI_E_INVALID) is cut into blocks of 64
 * ids, a block being its first id as a 32-bit word and then the gaps to the
 * next ids bit-packed at the list's gap width, then the block's weights
 * bit-packed at the list's weight width (the bit length of its largest
 * weight).  The blocks go where the placement puts the lists;
 * col and weights are read only during creation.  BFS, SSSP, CC and
 * PageRank scan packed lists with the edge-balanced variant (V5) whatever
 * the scheduler (BFS levels may also run bottom-up, see emogi_set_direction);
 * SSSP then reads each scanned list's packed weights whole.
 * Batched traversal decodes the same blocks.  The HBM tier is
 * EMOGI_E_UNSUPPORTED on packed graphs.
 * Nothing is leaked on failure; *out is set only on success. */
emogi_status_t emogi_graph_create(const uint64_t *row_ptr, uint64_t num_vertices,
                                  const void *col, uint32_t col_bytes,
                                  const uint32_t *weights, emogi_placement_t placement,
                                  uint32_t flags, emogi_graph_t *out);
emogi_status_t emogi_graph_destroy(emogi_graph_t g);
/* Bytes of the packed ids and of the packed weights (weight_bytes may be
 * NULL); both 0 for a graph created without EMOGI_F_PACK. */
emogi_status_t emogi_packed_bytes(emogi_graph_t g, uint64_t *id_bytes, uint64_t *weight_bytes);

/* Request unit R (bytes, power of two 32..4096) used to round list starts
 * down (Sec. 4.3.2).  Default 256: the smallest block that runs the MI355X
 * host link at its copy rate when read at random. */
emogi_status_t emogi_set_request_unit(emogi_graph_t g, uint32_t bytes);
emogi_status_t emogi_set_scheduler(emogi_graph_t g, int mode);
/* BFS levels enqueued per host wait.  Each level's kernels read the frontier
 * length the previous level left in device memory, so a batch needs no host
 * round trip between its levels (Sec. 4.2 launches one kernel per level and
 * the host checks for termination after each).  1: one level per wait, the
 * variant chosen per level; k > 1 (<= 64): k levels per wait with one
 * variant (the fixed one, else a workgroup per vertex below 2^24 edges and
 * the heuristic's pick for the whole graph above) and
 * pushes through the LDS-staged queue; 0 (default): 8 on graphs of fewer
 * than 2^24 edges, 1 above.  Always 1 when the scheduler records features
 * (EMOGI_SCHED_RECORD) or probes; under EMOGI_SCHED_LEARNED the batches stay
 * and the network picks the variant only of levels run one per host wait
 * (stats.levels_by_network counts them).  Results are identical. */
emogi_status_t emogi_set_level_batch(emogi_graph_t g, uint32_t levels);
/* SSSP distance band (near-far worklist): every vertex whose distance
 * improves is marked; a round expands, in ascending id order, the marked
 * vertices whose distance is below the current split, and when none is left
 * the split moves to the smallest marked distance + delta.  0 disables the
 * bands (every improved vertex is expanded in the next round).  Default 3.
 * Results are identical for any value; only the amount of re-expansion
 * changes. */
emogi_status_t emogi_set_sssp_delta(emogi_graph_t g, uint32_t delta);
/* Frontier order for BFS and CC label propagation: 0 appends pushes through
 * per-wave LDS segments (order unspecified); 1 (default) collects the next
 * frontier as a bitmap and lists it in ascending vertex id, so each level
 * reads neighbour lists in edge-array order.  SSSP always lists its marks.
 * Results are identical either way. */
emogi_status_t emogi_set_frontier_order(emogi_graph_t g, int ordered);
/* CC algorithm (both give every vertex the smallest id of its component):
 * EMOGI_CC_LABEL_PROPAGATION: all vertices start active and push their label
 *   over every list until nothing changes (the paper's workload, Sec. 5.4);
 * EMOGI_CC_SAMPLED_UNION_FIND (default): hook each vertex to its first two
 *   neighbours, compress, then read whole lists only for vertices outside
 *   the largest tree found (Afforest-style; far fewer list bytes). */
#define EMOGI_CC_LABEL_PROPAGATION 0
#define EMOGI_CC_SAMPLED_UNION_FIND 1
emogi_status_t emogi_set_cc_algorithm(emogi_graph_t g, int algorithm);
/* Loads the 5638 fp32 scheduler parameters (order W1,b1,W2,b2,W3,b3, row-major)
 * from host memory; NULL clears them (learned mode then uses the heuristic). */
emogi_status_t emogi_set_scheduler_weights(emogi_graph_t g, const float *params, size_t count);
/* The feature range the network was trained on: lo[16] and hi[16] (host).
 * A level whose features fall outside [lo, hi] in any component uses the
 * heuristic instead of the network (no extrapolation).  Both NULL: no check. */
emogi_status_t emogi_set_scheduler_range(emogi_graph_t g, const float *lo, const float *hi);

/* ---- scheduler network training (16 -> 64 -> 64 -> 6, ReLU, softmax
 *      cross-entropy, Adam; fp32 HIP kernels).  The worker-size trade-off of
 *      Sec. 4.3.1 and the GK/GU contrast of Sec. 5.3.1 motivate choosing the
 *      variant per level; the network is trained on per-level timings. ----
 * Device-pointer primitives (all arrays hipMalloc'd, row-major):
 *   params float[5638] (W1[64][16], b1[64], W2[64][64], b2[64], W3[6][64], b3[6]),
 *   X float[B][16], y int32[B] in 0..5, Z float[B][6], grad float[5638],
 *   loss float[1] (mean over the batch; may be NULL). */
emogi_status_t emogi_mlp_forward(const float *params, const float *X, uint32_t B, float *Z,
                                 void *stream);
emogi_status_t emogi_mlp_loss_grad(const float *params, const float *X, const int32_t *y,
                                   uint32_t B, float *grad, float *loss, void *stream);
/* One Adam step in place (m, v: float[5638] moment buffers; t counts from 1). */
emogi_status_t emogi_mlp_adam_step(float *params, const float *grad, float *m, float *v,
                                   uint32_t t, float lr, float beta1, float beta2, float eps,
                                   void *stream);
typedef struct {
    float lr, beta1, beta2, eps;
    uint32_t batch;   /* minibatch size */
    uint32_t epochs;
    uint64_t seed;    /* shuffling */
} emogi_train_config_t;
/* Whole training run on the GPU from host arrays: X float[N][16], y int32[N];
 * params (host, 5638 floats) holds the initial weights and receives the
 * trained ones; loss_history (host, `epochs` floats, may be NULL) gets the mean
 * minibatch loss per epoch.  Only full minibatches are used. */
emogi_status_t emogi_mlp_train(const float *X, const int32_t *y, uint32_t N,
                               const emogi_train_config_t *cfg, float *params,
                               float *loss_history);

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

/* BFS that allocates nothing, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same result as emogi_bfs: levels (device uint32[V], caller
 * owned) receives the level of every vertex, 0xFFFFFFFF when unreachable.
 * The same level kernels run top-down, 8 levels enqueued per host wait; the
 * variant is the fixed scheduler variant if one of V0..V4 is set, else a
 * workgroup per vertex.  Every device buffer it needs (two frontier queues,
 * the visited bitmap, level counters) lives in a 34 MiB array in the
 * library's device code, one per GPU, held until the process ends; the call
 * makes no hipMalloc, hipFree or other allocating call.
 * Limits and errors: V <= 2^22 (4,194,304) vertices, else EMOGI_E_INVALID;
 * packed graphs (EMOGI_F_PACK) EMOGI_E_UNSUPPORTED; src >= V or an output
 * that is not device memory EMOGI_E_INVALID; the graph's device must be the
 * current device (else EMOGI_E_INVALID).  All calls on one GPU share its
 * array, which keeps the last call's contents (each call clears what must
 * start at zero): calls that overlap on one GPU, from several threads or
 * streams, race and give undefined results.  Returns after the traversal has
 * completed; emogi_last_stats reports it (levels, edges, link bytes, times). */
emogi_status_t emogi_bfs_noalloc(emogi_graph_t g, uint64_t src, uint32_t *levels, void *stream);

/* PageRank (the fourth workload of Sec. 5.1), pull form on an undirected
 * graph (created with EMOGI_F_SYMMETRIC, else EMOGI_E_NOT_SYMMETRIC), in
 * fixed point so that every sum is exact: scores are uint64 with
 * `frac_bits` fractional bits (one = 2^frac_bits, 1 <= frac_bits <= 62) and
 * the damping factor is the integer damping_fixed = floor(damping * one),
 * which must be below one.  With deg(u) the list length of u:
 *   pr_0(v)     = floor(one / V)
 *   c(u)        = floor(pr(u) / deg(u))   (0 when deg(u) = 0)
 *   pr_{t+1}(v) = floor((one - damping_fixed) / V)
 *                 + floor(damping_fixed * sum over neighbours u of c(u) / one)
 * A vertex without neighbours passes nothing on.  Integer sums make the
 * result independent of the order of additions.  Runs `iters` iterations,
 * each streaming every neighbour list once (V5 chunks of all lists, the HBM
 * tier when set).  `scores`: device uint64[V], written with pr_iters.
 * Returns after the last iteration; stats count one level per iteration. */
emogi_status_t emogi_pagerank(emogi_graph_t g, uint32_t iters, uint32_t frac_bits, uint64_t damping_fixed,
                              uint64_t *scores, void *stream);

/* ---- batched multi-source traversal (the paper runs 64 sources per graph,
 *      Sec. 5.2; here up to 64 run together and each list read from host
 *      memory serves every source active at that vertex) ----
 * srcs     host uint64[n], 1 <= n <= 64, each < V (repeats allowed).
 * out      device uint32[n * V], source-major: out[s * V + v].
 * BFS gives levels, SSSP distances (weights required), per source exactly as
 * emogi_bfs / emogi_sssp would.  Level steps are captured in hipGraphs and
 * replayed on a private stream; the call returns when all sources finish. */
typedef struct {
    uint32_t hub_degree;      /* lists longer than this are scanned by a whole workgroup */
    uint32_t steps_per_graph; /* level steps per hipGraph replay (even, 2..32)             */
    uint32_t blocks_per_cu;   /* grid = 256 * blocks_per_cu workgroups (1..8)             */
    uint32_t use_graph;       /* 1: capture + replay hipGraphs, 0: launch steps directly   */
    uint32_t sssp_delta;      /* SSSP distance band shared by the batch's sources.  0: one
                                 band, every improvement expanded in the next step.  d > 0:
                                 a source whose distance at a vertex is not below the split
                                 waits there (one bit per vertex and source); when a step
                                 expands nothing the split moves to the smallest waiting
                                 distance + d and the waiting sources below it are listed
                                 (one pass over V).  Results do not depend on d.           */
} emogi_batch_params_t;

emogi_status_t emogi_bfs_batch(emogi_graph_t g, const uint64_t *srcs, uint32_t n, uint32_t *out,
                               void *stream);
emogi_status_t emogi_sssp_batch(emogi_graph_t g, const uint64_t *srcs, uint32_t n, uint32_t *out,
                                void *stream);
emogi_status_t emogi_set_batch_params(emogi_graph_t g, const emogi_batch_params_t *p);
emogi_status_t emogi_get_batch_params(emogi_graph_t g, emogi_batch_params_t *p);
/* Autotuner: runs the batched traversal (algo 0 = BFS, 1 = SSSP) for each
 * candidate parameter set, keeps the fastest on the handle and returns it.
 * `out` is scratch of n * V uint32 (device) and holds the last result.
 * `table` (may be NULL) receives up to `table_len` (params, ms) pairs. */
typedef struct {
    emogi_batch_params_t params;
    float ms;
} emogi_batch_trial_t;
emogi_status_t emogi_autotune_batch(emogi_graph_t g, int algo, const uint64_t *srcs, uint32_t n,
                                    uint32_t *out, void *stream, emogi_batch_params_t *best,
                                    emogi_batch_trial_t *table, uint32_t table_len);

/* ---- HBM tier of neighbour lists (the GPU-memory caching of graph data
 *      that Sec. 6 proposes to cut host-link traffic further) ----
 * Copies into GPU memory the neighbour lists (and weights) of the vertices of
 * highest degree (ties: lower id first): the longest prefix of that order
 * whose col_bytes (+4 with weights) bytes per edge fit in `budget_bytes`.
 * Every scan of such a list (all variants, sampled CC, batched traversals)
 * then reads GPU memory instead of the edge list; results are unchanged and
 * stats.tier_edges counts the edges so read.  Replaces any previous tier;
 * budget 0 removes it.  Synchronous (device-wide); the copy reads the lists
 * once from the edge list's placement.  *tier_vertices and *tier_bytes (each
 * may be NULL) receive the tier's size.  EMOGI_E_OOM_DEVICE when the tier
 * would not leave 256 MiB of device memory free (no tier is then kept). */
emogi_status_t emogi_set_hbm_tier(emogi_graph_t g, uint64_t budget_bytes, uint64_t *tier_vertices,
                                  uint64_t *tier_bytes);

/* BFS level direction (direction-optimizing BFS; Sec. 6 notes that a pull
 * over incoming lists keeps the same access pattern as the push over
 * outgoing ones, and on an undirected graph a vertex's list is both).
 * A top-down level expands the frontier's lists (Algorithm 1); a bottom-up
 * level makes every unvisited vertex with edges read its own list, one
 * 32-byte sector at a time, until it meets a vertex of the frontier, which
 * makes it a vertex of the next level.  Levels are identical either way.
 *   EMOGI_DIR_TOP_DOWN : every level top-down;
 *   EMOGI_DIR_AUTO     : (default) per level, the rule of Beamer, Asanovic
 *                        and Patterson (SC 2012): switch to bottom-up when
 *                        the frontier's edges exceed the unvisited vertices'
 *                        edges / alpha, back to top-down when the frontier
 *                        holds fewer than (vertices with edges) / beta
 *                        vertices (alpha, beta >= 1; 0 keeps the current value;
 *                        defaults 14 and 24);
 *   EMOGI_DIR_BOTTOM_UP: every level after the source's bottom-up.
 * Bottom-up levels run only on graphs created with EMOGI_F_SYMMETRIC,
 * with the ordered frontier, one level per host wait and a scheduler mode
 * other than EMOGI_SCHED_PROBE; elsewhere every level is top-down.  On
 * packed lists a bottom-up level decodes a vertex's first 8 ids, then its
 * blocks in turn.  stats.level_direction records each level. */
#define EMOGI_DIR_TOP_DOWN 0
#define EMOGI_DIR_AUTO 1
#define EMOGI_DIR_BOTTOM_UP 2
emogi_status_t emogi_set_direction(emogi_graph_t g, int mode, uint32_t alpha, uint32_t beta);

/* Create-time passes of the graph: milliseconds spent computing each
 * vertex's smallest incoming weight (EMOGI_F_WEIGHT_BOUND's GPU pass; 0 when
 * it was not computed).  The pass reads col and weights once over the link. */
emogi_status_t emogi_graph_setup_ms(emogi_graph_t g, double *in_min_ms);

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
