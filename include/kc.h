/*
 * kc.h -- exact k-clique counting on one AMD Instinct MI355X (gfx950).
 *
 * Method: Almasri, El Hajj, Nagi, Xiong, Hwu, "Parallel K-clique Counting on
 * GPUs", ICS 2022 (arXiv 2104.13209).  The problem (Sec. 1): given an undirected
 * simple graph G and an integer k, return the number of k-vertex subsets of V
 * whose vertices are pairwise adjacent.
 *
 * Pipeline behind this header:
 *   kc_orient   orient G into a DAG by degree, degeneracy, approximate
 *               degeneracy or colouring order (Sec. 3.1),
 *               filter edges and rebuild the CSR by histogram + exclusive scan;
 *   kc_list     list the k-cliques themselves (the orientation traversal);
 *   kc_count    traverse one search tree per root vertex (vertex-centric) or root
 *               edge (edge-centric) (Sec. 3.2) over the root's induced sub-graph
 *               encoded as bitsets (Sec. 2.4, 3.4), without pivoting (Fig. 2) or
 *               with pivoting (Fig. 3);
 *   kc_count_all  counts for every clique size at once (Sec. 2.3: pivoting counts
 *               all k in one traversal).
 *
 * Conventions for every entry point
 *   - Pointers inside kc_csr / kc_dag and the workspace are DEVICE pointers,
 *     allocated and freed by the caller; the library never allocates device
 *     memory in these calls and never frees caller memory.  Result pointers
 *     (kc_u128*, int32_t*) passed as separate arguments are HOST pointers.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on
 *     it; calls that return a value to the host synchronise that stream.
 *   - Every call returns a kc_status; no exception or abort crosses the ABI.
 *   - Vertex ids are int32 in [0, n); CSR offsets are int32 (nnz < 2^31).
 */
#ifndef KC_H
#define KC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KC_API __attribute__((visibility("default")))

/* Exact unsigned 128-bit count: value = lo + 2^64 * hi. */
typedef struct kc_u128 { uint64_t lo, hi; } kc_u128;

typedef enum kc_status {
    KC_OK = 0,
    KC_EINVAL = -1,        /* bad argument or malformed graph (when validated)   */
    KC_ENOMEM = -2,        /* workspace too small                                */
    KC_EOVERFLOW = -3,     /* count does not fit the result width                */
    KC_EDEVICE = -4,       /* a HIP runtime call failed                          */
    KC_ECANCELED = -5,     /* the caller's cancel flag stopped the count          */
    KC_EUNSUPPORTED = -6   /* graph exceeds a documented limit of this build     */
} kc_status;

enum { KC_ORDER_DEGREE = 0, KC_ORDER_DEGENERACY = 1, KC_ORDER_APPROX_DEGENERACY = 2, KC_ORDER_COLOR = 3 };
enum { KC_SCHEME_AUTO = 0, KC_SCHEME_VC = 1, KC_SCHEME_EC = 2 };

/* Largest out-degree whose roots keep their bitset rows on chip (LDS,
 * s x ceil(s/32) words).  Roots whose first vertex has a longer out-row ("wide
 * roots") are counted by kc_count and kc_count_all from rows in a global-memory
 * slab per wavefront (Sec. 3.3, 3.6 keep sub-graphs and stacks in pre-allocated
 * global memory), up to KC_MAX_DMAX_WIDE.  kc_count_local, the list-
 * intersection ablation and kc_batch_count stay within KC_MAX_DMAX and return
 * KC_EUNSUPPORTED beyond it. */
#define KC_MAX_DMAX 1024
#define KC_MAX_DMAX_WIDE 8192

/* Undirected input graph (Sec. 3.1 CSR): row_ptr[n+1], col[nnz], each row
 * strictly increasing, no self-loops, symmetric (u in row v iff v in row u).
 * Device pointers, read only. */
typedef struct kc_csr {
    int32_t n;
    int32_t nnz;               /* = 2m */
    const int32_t* row_ptr;
    const int32_t* col;
} kc_csr;

/* Oriented graph (DAG) written by kc_orient.  Vertices are RELABELLED by their
 * position in the orientation order: DAG vertex i is input vertex perm[i], and
 * every edge i -> j has i < j.  Out-lists are sorted ascending (Sec. 3.4 assigns
 * bit positions in a fixed sorted vertex order; with this labelling a root's
 * bitset rows are upper triangular).  Caller-allocated device arrays:
 *   row_ptr[n+1], col[m], src[m] (COO source of each edge, Sec. 3.1 hybrid
 *   CSR + COO for edge-centric roots), perm[n].
 * n, m, d_max (max out-degree), degeneracy (-1 for degree order) and order are
 * host fields filled by kc_orient. */
typedef struct kc_dag {
    int32_t n, m, d_max, degeneracy, order;
    int32_t* row_ptr;
    int32_t* col;
    int32_t* src;
    int32_t* perm;
} kc_dag;

/* Optional per-call measurements (host struct filled by kc_count / kc_count_all
 * when kc_opts.profile is non-NULL).  Times are GPU durations from HIP events
 * recorded on the call's stream around each phase.  nodes / word_ops are filled
 * only when kc_opts.collect_stats != 0, which runs a separately compiled,
 * slower variant of the traversal kernels that counts its work: nodes = search
 * tree nodes expanded by the traversal (intersections of a candidate set with
 * one adjacency row), word_ops = sum over those nodes of the root's bitset row
 * length in 32-bit words (pivot traversal: plus the |I| + 1 rows of W words
 * read to choose each node's pivot and form its P'). */
typedef struct kc_profile {
    float ms_classify;         /* root classification into light / heavy lists */
    float ms_light;            /* traversal kernel over light roots             */
    float ms_heavy;            /* traversal kernel over heavy roots             */
    float ms_total;            /* whole call, first to last kernel              */
    uint64_t nodes[2];         /* [0] light list, [1] heavy list               */
    uint64_t word_ops[2];
    int32_t light_roots;       /* roots in each list (after pruning)            */
    int32_t heavy_roots;
    /* Default (lane-walk) path only: per width list j (rows of 2^j words),
     * the launch duration, roots, expanded nodes and their bitset words. */
    float ms_width[6];
    int32_t roots_width[6];
    uint64_t nodes_width[6];
    uint64_t words_width[6];
    uint64_t iters_width[6];   /* wavefront rounds (checks + up to 8 lane steps) */
    uint64_t expand_width[6];  /* node expansions summed over lanes; expand /
                                  (64 x rounds) = expansions per lane and round */
    int32_t waves_width[6];    /* wavefronts launched                           */
    float busy_width[6];       /* mean wavefront busy time / launch span         */
    int32_t items_width[6];    /* subtrees handed between wavefronts (pair mode) */
    uint64_t cwords_width[6];  /* stats: k-cliques counted, each weighted by its
                                  root's bitset row words; summed over k' = 3 ..
                                  k-1 this is the unpruned Fig. 2 tree's word count
                                  (one node per k'-clique) */
} kc_profile;

/* Flags of kc_opts:
 * KC_OPT_NO_HANDOFF      wavefronts never hand subtrees to idle wavefronts;
 * KC_OPT_SINGLE_STREAM   every launch stays on the caller's stream (no side
 *                        stream for the widest root list, no helper launch):
 *                        for callers that already run many counts at once;
 * KC_OPT_NO_BITSETS      non-pivot counts without binary encoding (the
 *                        ablation of Sec. 4.3): candidate sets are sorted vertex
 *                        lists and each intersection binary-searches the members
 *                        in the branch vertex's out-list, one wavefront per root.
 *                        Same counts; KC_EUNSUPPORTED when (k - 2) lists of
 *                        d_max entries do not fit one wavefront's LDS. */
enum { KC_OPT_NO_HANDOFF = 1, KC_OPT_SINGLE_STREAM = 2, KC_OPT_NO_BITSETS = 4 };

/* Tuning options; NULL means defaults.  scheme: KC_SCHEME_*; width: lanes per
 * sub-wavefront group (1, 2, 4, 8, 16, 32 or 64; 0 = auto) (Sec. 3.5).
 * collect_stats and profile: see kc_profile.  flags: KC_OPT_* bits.
 * test_preload: added to the internal accumulator before counting; it exists
 * only so that tests can drive the 64-bit overflow path, and is 0 in normal use.
 * cancel: NULL, or the address of an int32 that the traversal kernels read while
 *   they run (device memory, or host memory allocated with hipHostMalloc and
 *   mapped into the device's address space, which any host thread may write).
 *   Once it holds a non-zero value the kernels stop taking work and the call
 *   returns KC_ECANCELED with no valid count; the caller owns the flag and
 *   resets it.  Kernels look at it when they start, every 32 wavefront rounds
 *   of a walk (non-pivot) or 32 tree nodes (pivot), and between roots, so a
 *   request takes effect within microseconds to milliseconds; calls that
 *   launch no traversal (k <= 2, k > d_max + 1) ignore it.
 * handoff_after, handoff_every: thresholds of the handoff between wavefronts
 *   (0 = defaults: a walk may hand subtrees over after 256 wavefront rounds on
 *   its current root or subtree and looks every 16 rounds; pivot trees after
 *   8192 nodes, 65536 for edge roots of at most 64 candidates, looking every
 *   64).  A value given here applies to every root list.  Lower values exist
 *   for tests and measurement; counts never depend on them. */
typedef struct kc_opts {
    int32_t scheme;
    int32_t width;
    int32_t collect_stats;
    int32_t flags;
    uint64_t test_preload;
    kc_profile* profile;
    const volatile int32_t* cancel;
    int32_t handoff_after;
    int32_t handoff_every;
} kc_opts;

/* Bytes of device workspace kc_orient needs for this input size and order. */
KC_API size_t kc_orient_workspace(int32_t n, int32_t nnz, int32_t order);

/* Orient g (Sec. 3.1).  order: KC_ORDER_DEGREE (edge u->v iff (deg u, u) <
 * (deg v, v)), KC_ORDER_DEGENERACY (k-core removal order from GPU peeling in
 * level-synchronous rounds; ties inside a round by id) or
 * KC_ORDER_APPROX_DEGENERACY (a relaxation of k-core, among the criteria of
 * Sec. 2: in rounds, every remaining vertex whose current degree is at most 1.1
 * times the remaining graph's average degree, i.e. 10 deg L <= 11 D for L
 * vertices of degree sum D, leaves at once; order by (round, id); far fewer
 * rounds than exact peeling, out-degrees at most 2.2 times the degeneracy;
 * dag->degeneracy is -1 as for degree order) or KC_ORDER_COLOR (graph
 * colouring, also among the criteria of Sec. 2: the greedy first-fit colouring
 * in decreasing order of the priority SplitMix64(v) (its output function applied
 * to v + 0x9E3779B97F4A7C15; ties by the larger id), computed by Jones-Plassmann
 * rounds; order by (colour, id), so every edge leaves its lower colour;
 * degeneracy -1; out-degrees are not bounded by the degeneracy and can exceed
 * KC_MAX_DMAX on skewed graphs).  Fills *out (device
 * arrays must hold n+1, m, m and n int32 with m = nnz/2) and its host fields;
 * synchronises `stream`.  validate != 0 first checks that g is a sorted simple
 * symmetric CSR and returns KC_EINVAL if not; with validate == 0 a malformed
 * graph gives an unspecified DAG.  Returns KC_ENOMEM if ws_bytes is below
 * kc_orient_workspace(). */
KC_API int32_t kc_orient(const kc_csr* g, int32_t order, kc_dag* out, void* ws,
                         size_t ws_bytes, int32_t validate, void* stream);

/* Bytes of device workspace kc_count / kc_count_all need for this DAG. */
KC_API size_t kc_count_workspace(const kc_dag* d, int32_t k, int32_t pivot, const kc_opts* o);

/* Number of k-cliques of the DAG's graph into *count (host).
 *   pivot == 0: graph-orientation traversal (Fig. 2); the result is a 64-bit
 *               count (count->hi == 0) and KC_EOVERFLOW is returned when the true
 *               count is 2^64 or more.
 *   pivot != 0: hybrid pivoting traversal (Fig. 3, Sec. 2.3); 128-bit count,
 *               KC_EOVERFLOW at 2^128 or more.
 * k < 1 is KC_EINVAL; k = 1 gives n and k = 2 gives m.  Synchronises `stream`.
 * Deep non-pivot counts run the widest root list on an auxiliary stream of the
 * library's own (fork and join by events on `stream`) unless KC_OPT_SINGLE_STREAM
 * is set; wavefronts hand work to idle ones through the workspace's queues unless
 * KC_OPT_NO_HANDOFF is set.  KC_EDEVICE is returned when such a queue stops making
 * progress for 20 s (no count is valid then).  One workspace serves one call at a
 * time.  Wide roots (see KC_MAX_DMAX) run after the others, one wavefront each;
 * KC_EUNSUPPORTED when d_max exceeds KC_MAX_DMAX_WIDE. */
KC_API int32_t kc_count(const kc_dag* d, int32_t k, int32_t pivot, kc_u128* count, void* ws,
                        size_t ws_bytes, const kc_opts* o, void* stream);

/* Per-vertex counts: local[v] = number of k-cliques that contain input vertex v
 * (DEVICE array of n uint64, indexed by INPUT vertex id, overwritten).  The sum
 * over v is k times kc_count's result.
 *   pivot == 0: the graph-orientation traversal (Fig. 2) finds each k-clique
 *     once, at a node whose path P has k - 1 vertices and whose candidate set is
 *     I; every vertex of P gains |I| and every member of I gains 1.
 *   pivot != 0: the pivoting traversal (Fig. 3); a leaf with holds H and pivots
 *     P stands for C(|P|, k - |H|) k-cliques (Sec. 2.3); every hold gains that
 *     many and every pivot C(|P| - 1, k - |H| - 1).
 * k = 1 gives 1 for every vertex, k = 2 the degree.  Uses kc_count_workspace()
 * bytes of workspace for the same (dag, k, pivot, opts); honours kc_opts.scheme
 * and cancel.  Returns KC_EOVERFLOW if a vertex's count reaches 2^64.  Deep
 * counts on skewed graphs are slower than kc_count: every tree stays on the
 * wavefront that took its root.  KC_EUNSUPPORTED when d_max exceeds KC_MAX_DMAX.
 * Synchronises `stream`. */
KC_API int32_t kc_count_local(const kc_dag* d, int32_t k, int32_t pivot, uint64_t* local, void* ws,
                              size_t ws_bytes, const kc_opts* o, void* stream);

/* k-clique listing (the orientation traversal of Fig. 2 with a listing leaf:
 * a node whose path P has k - 1 vertices and candidate set I stands for the
 * cliques P + {w}, w in I).  Writes up to `cap` cliques into the DEVICE array
 * cliques[cap * k], one row of k INPUT vertex ids per clique in ascending
 * orientation rank (the clique's lowest-ranked vertex first), and the number of
 * k-cliques into *total (host).  When *total > cap, the first cap rows hold cap
 * of them (which ones is unspecified: rows are reserved by concurrent
 * wavefronts); otherwise the first *total rows hold every k-clique once, in an
 * unspecified row order.  k = 1 lists the vertices, k = 2 the edges.  Uses
 * kc_count_workspace(d, k, 0, o) bytes; honours kc_opts.scheme and cancel.
 * KC_EINVAL for k < 1, cap < 0 or a NULL array with cap > 0; KC_EUNSUPPORTED when
 * d_max exceeds KC_MAX_DMAX.  Synchronises `stream`. */
KC_API int32_t kc_list(const kc_dag* d, int32_t k, int32_t* cliques, int64_t cap, uint64_t* total, void* ws,
                       size_t ws_bytes, const kc_opts* o, void* stream);

/* Size of the fixed device scratch array behind kc_count_noalloc (64 MiB per
 * GPU the library runs on, held until the process ends). */
#define KC_NOALLOC_SCRATCH_BYTES (64u << 20)

/* kc_count without a caller workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, result and statuses as kc_count; the
 * workspace is a file-scope device array of KC_NOALLOC_SCRATCH_BYTES, one per
 * GPU, whose address is looked up once per device on the first call made with
 * that device current.  The call allocates nothing (no hipMalloc, no stream or
 * event creation): it always runs single-stream (KC_OPT_SINGLE_STREAM is
 * forced) and ignores kc_opts.profile and collect_stats.  Returns KC_ENOMEM when
 * kc_count_workspace() for this DAG exceeds KC_NOALLOC_SCRATCH_BYTES (about
 * 16 bytes per root plus 5 MB: non-pivot counts of graphs up to roughly 3.8M
 * edges).  Every call on one GPU shares that GPU's array and leaves its contents
 * behind (each call re-initialises what it reads): calls that overlap in time on
 * the same GPU, from any thread or stream, race and must be serialised by the
 * caller.  Synchronises `stream`. */
KC_API int32_t kc_count_noalloc(const kc_dag* d, int32_t k, int32_t pivot, kc_u128* count,
                                const kc_opts* o, void* stream);

/* counts[j] = number of j-cliques for j = 0..cap (host array of cap+1), with
 * counts[0] = 1 (the empty clique), counts[1] = n, counts[2] = m; *omega = the
 * largest j with a j-clique (the clique number).  pivot != 0 uses one pivoting
 * traversal for every size (Sec. 2.3).  pivot == 0 runs the graph-orientation
 * traversal (Fig. 2) once per size, k = 3, 4, ..., until a size has no clique
 * (at most d_max + 1), so its cost is one kc_count per size up to omega + 1
 * whatever cap is.  Returns KC_EINVAL if cap < 2, KC_EOVERFLOW if a count
 * needs more than 128 bits and KC_EUNSUPPORTED when d_max exceeds
 * KC_MAX_DMAX_WIDE.  Synchronises `stream`. */
KC_API int32_t kc_count_all(const kc_dag* d, int32_t pivot, kc_u128* counts, int32_t cap,
                            int32_t* omega, void* ws, size_t ws_bytes, const kc_opts* o,
                            void* stream);

/* ------------------------------------------------------------- batched */

/* Many independent graphs packed into one CSR (device pointers): graph g owns
 * vertices [voff[g], voff[g+1]) and its rows reference only its own vertices.
 * max_degree bounds every vertex degree (it sizes the radix sort on the host, so
 * no value has to be read back).  max_graph_edges bounds the undirected edge
 * count of every graph (0 = unknown): under degree orientation a vertex with t
 * out-neighbours has t + 1 vertices of degree >= t in its graph, so
 * t <= sqrt(2 max_graph_edges); the smaller of that and max_degree bounds every
 * root candidate set. */
typedef struct kc_batch {
    int32_t ngraphs;
    int32_t n;                 /* total vertices = voff[ngraphs]        */
    int32_t nnz;               /* total CSR entries                     */
    int32_t max_degree;
    const int32_t* row_ptr;    /* [n+1]                                 */
    const int32_t* col;        /* [nnz]                                 */
    const int32_t* voff;       /* [ngraphs+1]                           */
    int32_t max_graph_edges;   /* largest m of one graph (0 = unknown)  */
} kc_batch;

#define KC_BATCH_MAX_BUCKETS 8

/* Execution plan by graph size: graphs with voff[g+1] - voff[g] <= n_hi[b] (the
 * first such bucket b, n_hi ascending) are counted with root scheme scheme[b]
 * (KC_SCHEME_VC / KC_SCHEME_EC) and traversal width[b]: 0 (or 1) = the lane walk
 * (one lane per subtree), 2, 4, 8, 16 or 32 = sub-wavefront groups of that many
 * lanes sharing each subtree (Sec. 3.5; lists of at most 64 candidates use
 * groups of at most 8 lanes, wider lists of at least 4).  Graphs above the last
 * bound use the last bucket.  Written by the autotuner; NULL = vertex roots and
 * the lane walk for every graph. */
typedef struct kc_batch_plan {
    int32_t nbuckets;
    int32_t n_hi[KC_BATCH_MAX_BUCKETS];
    int32_t scheme[KC_BATCH_MAX_BUCKETS];
    int32_t width[KC_BATCH_MAX_BUCKETS];
} kc_batch_plan;

/* Bytes of device workspace kc_batch_count needs. */
KC_API size_t kc_batch_workspace(const kc_batch* b, int32_t k);

/* Per-graph k-clique counts of a packed batch (non-pivot traversal, degree
 * orientation), written to the DEVICE array counts[2*ngraphs] as {lo, hi}
 * pairs.  Everything runs on `stream` with no host synchronisation, no device
 * allocation and no memset, so the call can be captured in a HIP graph and
 * replayed.  A per-graph overflow past 2^64 leaves a non-zero hi word (the
 * caller's 64-bit check).  Returns KC_EINVAL for k < 1, bad sizes or a plan
 * with an unknown scheme or width, KC_ENOMEM for a short workspace, KC_EUNSUPPORTED if
 * the out-degree bound min(max_degree, sqrt(2 max_graph_edges)) exceeds
 * KC_MAX_DMAX (rows could not be bitset-encoded). */
KC_API int32_t kc_batch_count(const kc_batch* b, int32_t k, uint64_t* counts, void* ws, size_t ws_bytes,
                              const kc_batch_plan* plan, void* stream);

/* ------------------------------------------------------------- serving */

/* A query server over oriented graphs that stay resident on the device
 * (continuous batching).  Queries (graph, k, pivot) are admitted in arrival
 * order when one of `slots` workers is free, the query's workspace
 * (kc_count_workspace) fits in the server's device arena of `mem_budget` bytes,
 * and (unless no other query runs) the estimated LDS of the admitted queries
 * stays within the device's LDS (per query: one wavefront's LDS for its widest
 * root list or pivot kernel times the wavefronts it launches, at most one per
 * root); admitted queries run concurrently, one HIP stream per worker, so work of
 * queries that arrive while others run overlaps on the device.  A query that
 * could never fit the arena completes at once with status KC_ENOMEM.
 * Ownership: the server allocates its arena and streams in kc_server_create and
 * frees them in kc_server_destroy (the only entry points that allocate device
 * memory); the kc_dag arrays stay owned by the caller and must outlive the
 * server.  Thread-safe: submit and wait may be called from any host thread. */
typedef struct kc_server kc_server;

typedef struct kc_query_result {
    uint64_t ticket;
    int32_t graph, k, pivot;
    int32_t status;            /* kc_count's status for this query            */
    kc_u128 count;
    double t_submit;           /* host steady-clock seconds                   */
    double t_start;            /* admitted and started on a worker            */
    double t_done;             /* result on the host                          */
    uint64_t workspace;        /* bytes admitted against the arena            */
    uint64_t lds;              /* estimated resident LDS bytes admitted       */
} kc_query_result;

KC_API int32_t kc_server_create(const kc_dag* dags, int32_t ndags, int32_t slots, uint64_t mem_budget,
                                kc_server** out);
/* Enqueue a query; *ticket identifies it.  Never blocks on the device.  Returns
 * KC_ECANCELED once kc_server_destroy has begun. */
KC_API int32_t kc_server_submit(kc_server* s, int32_t graph, int32_t k, int32_t pivot, uint64_t* ticket);
/* Block until the query is done and return its result (each ticket once). */
KC_API int32_t kc_server_wait(kc_server* s, uint64_t ticket, kc_query_result* res);
/* Shut the server down: queries never admitted end with status KC_ECANCELED
 * (threads blocked on them in kc_server_wait wake up and receive that result),
 * admitted queries run to completion, and the server's memory and streams are
 * freed only after every thread inside kc_server_wait has returned.  No call on
 * `s` may begin after kc_server_destroy has returned. */
KC_API int32_t kc_server_destroy(kc_server* s);

/* Static text for a status code. */
KC_API const char* kc_strerror(int32_t status);

/* Release the library's process-wide pools (the auxiliary streams of deep
 * non-pivot counts and the timing events of profiled calls, created on first
 * use).  The library also does this at process exit, before the HIP runtime's
 * own teardown; calling it earlier is allowed when no call is in flight, and
 * later calls simply create new pool entries. */
KC_API void kc_shutdown(void);

#ifdef __cplusplus
}
#endif
#endif /* KC_H */
