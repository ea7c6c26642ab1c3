/*
 * gc.h -- C ABI of the MI355X group-closeness library (libgc.so).
 *
 * Method: Greedy++ for group closeness maximisation (Bergamini, Gonser,
 * Meyerhenke, "Scaling up Group Closeness Maximization").  On a connected,
 * undirected, unweighted graph G = (V, E) (Section 2) the library picks k nodes
 * greedily, each time adding the node with the largest marginal gain
 *     g(v, S) = F(S) - F(S u {v}),   F(S) = sum_{w in V} d(S, w),
 * where d(S, w) = min_{s in S} d(s, w) (Section 2).  F is the integer group
 * farness: n times the paper's f(S) = 1/c(S) with c(S) = n / sum d(S, v)
 * (Section 2), and the objective of the ILP of Section 5.  Gains are computed
 * exactly by BFS from v pruned to nodes w with d(v, w) < d(S, w) (Section 4.1);
 * gains of earlier rounds are upper bounds that let the greedy loop skip
 * candidates (Section 4.2, valid by the supermodularity lemma of Section 3.2).
 *
 * Weighted graphs (gc_load_csr_weighted): every edge has an integer length
 * 1..255 and d is the SSSP distance (Section 2 names SSSP in general, BFS
 * being the unit-length case); the pruning of Section 4.1 and the lazy loop of
 * Section 4.2 hold unchanged.  Each candidate's search runs inside one
 * workgroup as a bucketed label-correcting search (delta-stepping).
 *
 * Conventions for every function
 *  - Return value: GC_OK (0) or a negative gc_status.  On error no output is
 *    written; gc_last_error() gives a message (thread-local).
 *  - d_* arguments are device pointers (HIP global memory) owned by the caller;
 *    h_* arguments are host pointers owned by the caller.  The library never
 *    allocates device memory: all device scratch lives in a caller-supplied
 *    workspace of at least gc_workspace_size() bytes that was prepared once by
 *    gc_workspace_init().  Every call returns the workspace to its prepared
 *    state, so it can be reused by later calls on the same stream.  Calls that
 *    share one workspace must not overlap in time (use one stream).
 *  - Work is enqueued on `stream`.  Calls with h_* outputs synchronise the
 *    stream before returning; calls with only d_* outputs are asynchronous.
 *  - Distances d(S, .) are stored as uint8 (dist_bytes = 1, INF = 255) or
 *    uint16 (dist_bytes = 2, INF = 65535); on a weighted graph as int32
 *    (dist_bytes = 4, INF = 2^31 - 1).  A distance array that is INF
 *    everywhere stands for S = {} .
 *  - Node ids are int32 in [0, n); ties between equal gains or equal farness
 *    always go to the smallest node id.
 *  - Watchdogs, read by gc_load_csr / gc_load_csr_weighted from the
 *    environment (default: none): GC_LEVEL_CAP=L makes a call whose BFS needs
 *    more than L levels fail with GC_EDEVICE; GC_ROUND_CAP=R abandons a
 *    weighted search after R near-list rounds, and gc_closest_node,
 *    gc_topk_closeness and gc_greedy_group then fail with GC_EDEVICE (the
 *    asynchronous weighted calls cannot report it; their outputs are then
 *    undefined).  Every kernel still ends normally; after GC_EDEVICE the
 *    distance array and F of the call are undefined and the workspace must be
 *    prepared again with gc_workspace_init.
 */
#ifndef GC_H
#define GC_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gc_status {
    GC_OK = 0,
    GC_EINVAL = -1,        /* bad argument, malformed CSR, k or node out of range */
    GC_ENOTSYM = -2,       /* adjacency is not symmetric (graph not undirected) */
    GC_EDISCONNECTED = -3, /* graph has more than one connected component */
    GC_ERANGE = -4,        /* a distance does not fit the chosen dist_bytes */
    GC_EWORKSPACE = -5,    /* workspace missing, too small or not initialised */
    GC_ENOMEM = -6,        /* host allocation failed */
    GC_EDEVICE = -7        /* a HIP runtime call failed */
} gc_status;

/* gc_load_csr flags */
#define GC_VALIDATE 0x1u /* check the CSR contract (default; strongly advised) */
#define GC_DIRECTED 0x2u /* rows are out-neighbour lists of a strongly connected
                            directed graph (Section 2); d(S, w) is measured along
                            the arcs, and validation checks strong connectivity
                            instead of symmetry */

/* candidate orders for the lazy greedy loop (gc_opts.order) */
#define GC_ORDER_PLAIN 0   /* ascending node id, the scan of the paper's while-loop */
#define GC_ORDER_CELF 1    /* stale gain descending, then id ascending */
#define GC_ORDER_LEARNED 2 /* MLP-predicted gain (capped by the stale gain) descending */

typedef struct gc_graph gc_graph; /* opaque; borrows the caller's device CSR */

/*
 * Options for gc_greedy_group.  Zero-initialise and set what you need;
 * a NULL opts pointer means all defaults (plain order, width 64, block 64).
 */
typedef struct gc_opts {
    int32_t order;          /* GC_ORDER_* */
    int32_t bitset_width;   /* sources per bit-parallel BFS: 64 (0 = default 64) */
    int32_t block;          /* rounds >= 2: candidates evaluated between two
                               threshold updates (0 = bitset_width); the picks
                               never depend on it */
    int32_t nprefix;        /* resume: the first nprefix picks are given */
    const int32_t *h_prefix;/* host, nprefix distinct ids (a previous run's pick
                               order); a repeated id gives GC_EINVAL */
    const void *d_mlp;      /* GC_ORDER_LEARNED: device inference block made by
                               gc_mlp_pack(); NULL otherwise */
    int32_t debug_checks;   /* 1: re-check F(S) == sum_w d(S,w) after every pick */
    int32_t block_growth;   /* each further launch of a round takes this many
                               times the block of the one before, up to
                               16 x block (1..8; 0 = default 2) */
    /* optional logging of every exact evaluation (host buffers, may be NULL):
       round, node, gain and the 8 MLP features at evaluation time */
    int64_t log_capacity;
    int32_t *h_log_round;
    int32_t *h_log_node;
    int64_t *h_log_gain;
    float *h_log_feat;      /* log_capacity x 8 */
    int64_t *h_log_count;   /* out: entries written (may exceed capacity: the rest dropped) */
    /* bitGreedy++ (Section 4.3 with the lazy loop): exact gains by the
       bit-vector sum from a buffer gc_bits_prepare filled (NULL: pruned BFS).
       bits_bytes: the size given to gc_bits_prepare.  Plain and CELF orders;
       uint8 distances (GC_ERANGE if ecc(s_1) > 254). */
    const void *d_bits;
    size_t bits_bytes;
    int32_t bits_levels;
    /* early exit inside the candidates' pruned BFS (a BFScut-style bound,
       Section 3.1, on the pruned BFS of Section 4.1), first gain round only:
       1 = on.  The early_exit_seed candidates of largest degree (0: 1024) are
       evaluated first, exactly; every other candidate of the round stops as
       soon as g_l + e_l + T[l+1] cannot beat their best, where g_l is its
       gain over the nodes claimed up to distance l, e_l the adjacency entries
       of those at distance l, and T[j] = sum_w max(0, d(S,w) - j - 1); its
       bound becomes its stale gain.  The picks never change; the evaluation
       counts of later rounds do.  Pruned-BFS gains only (not with d_bits). */
    int32_t early_exit;
    int32_t early_exit_seed;
} gc_opts;

/* Counters filled by gc_greedy_group (all optional). */
typedef struct gc_stats {
    int64_t evals_total;    /* exact gain evaluations, all rounds */
    int64_t evals_round1;   /* evaluations in the first round after s_1 (n-1) */
    int64_t evals_later;    /* evaluations in rounds >= 2 */
    int64_t edges_alg;      /* sum over evaluations of sum_{w in V(v)} deg(w) */
    int64_t visited;        /* sum over evaluations of |V(v)| */
    int64_t gain_launches;  /* gain-kernel launches */
    int64_t closest_sources;/* sources that entered a closeness BFS in gc_closest_node */
    int32_t dist_bytes;     /* width chosen for d(S,.) */
    int32_t ecc_s1;         /* eccentricity of the first pick */
    double ms_total;        /* wall time of the call (host clock) */
    double ms_closest;      /* finding s_1 */
    double ms_round1;       /* first gain round */
    double ms_later;        /* gain rounds >= 2 incl. selection */
    double ms_update;       /* d(S,.) updates */
    double ms_mlp;          /* feature + MLP inference (learned order) */
    /* word-level work of the gain launches (one frontier entry is a node
     * reached by some of the 64 sources of a batch at one level; see
     * gc_gain_words) */
    int64_t entries_word;   /* frontier entries, all levels */
    int64_t entries_root;   /* of which root entries (level 0) */
    int64_t entries_last;   /* of which entries of the last level (not expanded) */
    int64_t edges_word;     /* adjacency entries expanded (levels before the last) */
    int64_t edges_last;     /* adjacency entries of the last level's entries */
    int64_t touched_word;   /* (batch, node) records the gain launches touched */
    double ms_gain_gpu;     /* GPU time of the gain launches (HIP events), all rounds;
                             * measured only while gc_timing_enable(1) is in force */
    int64_t mlp_launches;   /* feature + MLP scoring launches (learned order) */
    int64_t bits_words;     /* bitGreedy++: 64-bit row words the bit-vector gains read */
    int64_t *h_evals_per_round; /* optional, caller-owned, k entries */
    int64_t cut_evals;      /* evaluations stopped by the early exit (gc_opts.early_exit) */
} gc_stats;

/* ---------------------------------------------------------------- graph --- */

/*
 * gc_load_csr -- wrap a device CSR as a graph handle (Section 2: connected,
 * undirected, unweighted G).
 *   n          node count, 1 <= n < 2^31
 *   nnz        entries of d_col_idx = 2|E| (each undirected edge stored twice)
 *   d_row_ptr  device int32[n+1], d_row_ptr[0] = 0, d_row_ptr[n] = nnz
 *   d_col_idx  device int32[nnz], each row strictly ascending
 *   flags      GC_VALIDATE: check the CSR on the host -- GC_EINVAL for a bad
 *              row_ptr, an id out of range, an unsorted row, a self-loop or a
 *              duplicate; GC_ENOTSYM for a missing reverse edge;
 *              GC_EDISCONNECTED if not connected.  GC_DIRECTED: a directed
 *              graph (no symmetry check; GC_EDISCONNECTED unless strongly
 *              connected); every call then follows arcs out of a row.
 *   stream     used for the copies: the CSR is copied to the host once (the
 *              degree order and the balls of nearby nodes that batch the
 *              closeness search are built there; host memory 4(n + nnz)
 *              bytes while loading)
 *   out        receives the handle (free with gc_free_graph)
 * The handle borrows the two device arrays: they must stay valid and
 * unchanged until gc_free_graph.  The handle may be used from several host
 * threads at once if each uses its own workspace.
 */
int gc_load_csr(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                uint32_t flags, hipStream_t stream, gc_graph **out);

/*
 * gc_load_csr_weighted -- as gc_load_csr, for a graph whose edges have
 * integer lengths (Section 2: distances are SSSP distances).
 *   d_weight   device uint8[nnz]: the length of the edge of each CSR entry,
 *              1..255; for an undirected graph both entries of an edge hold
 *              the same length.  Borrowed like the CSR arrays.
 *   n          1 <= n < 2^23 (GC_ERANGE otherwise), so that every distance,
 *              at most 255 (n - 1), fits int32
 *   flags      as for gc_load_csr; GC_VALIDATE also checks the lengths:
 *              GC_EINVAL for a length 0, GC_ENOTSYM for an undirected edge
 *              whose two entries differ
 * The lengths are copied to the host once (nnz bytes).  On the handle:
 * gc_closest_node, gc_topk_closeness, gc_update_dist and gc_marginal_gains
 * take int32 distances (dist_bytes = 4); gc_greedy_group takes the plain or
 * CELF order without bit vectors, early exit or evaluation log; the
 * bit-vector calls, gc_marginal_gains_noalloc, gc_gain_words and
 * gc_node_features give GC_EINVAL.  Read here: GC_WDELTA and
 * GC_WDELTA_CLOSE (the bucket widths of the gain and closeness searches;
 * defaults twice the largest length, and a sixteenth of the mean distance
 * from the first node the closeness search takes), GC_WSLOTS (gain searches
 * in flight, default 8 per compute unit within the record budget
 * GC_VIS_BUDGET_MB), GC_WCLOSE_SLOTS and GC_WCLOSE_THREADS (closeness
 * searches in flight and their workgroup size, default 256 and 1024).  None
 * changes a result.
 */
int gc_load_csr_weighted(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                         const uint8_t *d_weight, uint32_t flags, hipStream_t stream, gc_graph **out);
void gc_free_graph(gc_graph *g);
int32_t gc_graph_n(const gc_graph *g);
int64_t gc_graph_nnz(const gc_graph *g);

/*
 * gc_tuning -- launch shapes of the device-wide engine for one graph.  No
 * field changes any result (groups, farness, gains, evaluation counts, word
 * counters aside from the batching of the closeness search): they decide only
 * how the work is spread over the GPU, so a tuner may pick them per graph.
 * gc_load_csr sets them from the environment (GC_UNROLL, GC_UNROLL_SMALL,
 * GC_MIN_EDGES, GC_MIN_EDGES_SMALL, GC_LEVEL_WGS) or to the defaults.
 */
typedef struct gc_tuning {
    int32_t unroll;           /* adjacency entries per thread per step in
                               * launches of > 1024 sources: 4, 8 or 16 */
    int32_t unroll_small;     /* the same for launches of <= 1024 sources and
                               * the d(S,.) updates: 4 or 8 */
    int32_t min_edges;        /* adjacency entries per workgroup before a level
                               * takes more workgroups, large launches (>= 16) */
    int32_t min_edges_small;  /* the same for small launches (>= 16) */
    int32_t level_wgs_per_cu; /* workgroups per CU of a level kernel, 1..64 */
    int32_t reserved[3];      /* zero */
} gc_tuning;

/* gc_get_tuning -- the handle's current shapes into *out (GC_EINVAL on NULL). */
int gc_get_tuning(const gc_graph *g, gc_tuning *out);
/* gc_set_tuning -- replace them; GC_EINVAL (nothing changed) if a field is
 * out of range.  Not while another call on the same handle is running. */
int gc_set_tuning(gc_graph *g, const gc_tuning *t);

/* ------------------------------------------------------------ workspace --- */

/*
 * gc_workspace_size -- bytes of device workspace needed by every call below
 * for graph g and the given bit-parallel width (64, or 0 for the default).
 * GC_EINVAL for another width.
 */
int gc_workspace_size(const gc_graph *g, int32_t bitset_width, size_t *bytes);

/*
 * gc_workspace_init -- prepare a workspace of ws_bytes >= gc_workspace_size()
 * bytes for graph g (zero-fills it and stamps a header).  Asynchronous on
 * stream.  Needed once per (workspace, graph); the library's calls keep it
 * prepared.  GC_EWORKSPACE if it is too small.
 */
int gc_workspace_init(const gc_graph *g, void *d_ws, size_t ws_bytes, hipStream_t stream);

/* ----------------------------------------------------------- operations --- */

/*
 * gc_closest_node -- s_1 = argmin_v F({v}), the node of maximum closeness
 * c(v) = (n-1)/sum_w d(v,w) (Section 2), first line of the memory-efficient
 * greedy (Appendix, Algorithm "mem-greedy").  Found as in top-k closeness with
 * k = 1 (Section 3.1, Algorithm "topk"): a level-1 bound drops most nodes, the
 * rest run as BFS in batches of 64 nearby nodes (balls seeded by decreasing
 * degree), each BFS cut as soon as a lower bound on its farness exceeds the
 * best farness found.  Ties go to the smallest id.
 *   h_node     host out: s_1
 *   h_farness  host out: F({s_1})
 * Synchronises the stream.  GC_ERANGE for graphs with more than 2^20 nodes
 * or 2^25 adjacency entries (the largest class this search has been run
 * on; the same limit holds for gc_topk_closeness and for gc_greedy_group
 * without a prefix).  Weighted graphs: one search per node in decreasing
 * degree order (the first alone), each stopped once the nodes it has settled
 * below theta and theta for every other node add up to more than the best
 * farness found; GC_EDISCONNECTED if a finished search missed a node.
 */
int gc_closest_node(const gc_graph *g, void *d_ws, size_t ws_bytes, hipStream_t stream,
                    int32_t *h_node, int64_t *h_farness);

/*
 * gc_topk_closeness -- the k nodes of maximum closeness, i.e. of least F({v}),
 * in increasing (F({v}), v) order (top-k closeness, Section 3.1, Algorithm
 * "topk", for general k; ties go to the smaller id).  The same search as
 * gc_closest_node with the k-th best farness found so far as the cut
 * threshold; no BFS is cut before k farness values are known.
 *   k          1..n (else GC_EINVAL)
 *   h_nodes    host out, k entries
 *   h_farness  host out, k entries: F({h_nodes[i]})
 * Uses the workspace as gc_closest_node does; synchronises the stream.
 * Outputs are untouched on error.
 */
int gc_topk_closeness(const gc_graph *g, int32_t k, void *d_ws, size_t ws_bytes, hipStream_t stream,
                      int32_t *h_nodes, int64_t *h_farness);

/*
 * Bit-vector gains (Section 4.3, bit-parallel group closeness; the gain
 * evaluation of bitGreedy++).  b^i_u is the set of nodes within distance i of
 * u as an n-bit row; the gain of u is the sum over i of |b^i_u AND NOT b^i_S|
 * (the theorem of Section 4.3).  The rows of every level are stored: n * n
 * bits per level, so this is for graphs with n up to about 10^5 and a small
 * diameter.
 *
 * gc_bits_size -- bytes of a caller buffer holding `levels` levels (2..256)
 *   plus the b^i_S rows and a counter block.
 * gc_bits_prepare -- compute b^0 (one bit per row), b^1, ... into d_bits until
 *   a level equals the one before (the fixed point; as many levels as the
 *   diameter + 1).  h_levels: the stored levels, the last the fixed point.
 *   GC_EWORKSPACE if the buffer holds too few levels.  Synchronises once per
 *   level.  The rows depend on the graph only.
 * gc_bits_gains -- g(v, S) for the count candidates in d_cand (device int32,
 *   ids in [0, n)) into d_gain (device int64), for the S whose distances
 *   d_dist holds (uint8 only, dist_bytes = 1; INF everywhere is S = {}), from
 *   a buffer gc_bits_prepare filled with `levels` levels, passed with the same
 *   `bytes` (the b^i_S rows sit after as many levels as that size holds).  The
 *   same values as gc_marginal_gains.  Synchronises once (max d(S,.)).
 */
int gc_bits_size(const gc_graph *g, int32_t levels, size_t *bytes);
int gc_bits_prepare(const gc_graph *g, void *d_bits, size_t bytes, hipStream_t stream, int32_t *h_levels);
int gc_bits_gains(const gc_graph *g, const void *d_bits, size_t bytes, int32_t levels, const void *d_dist,
                  int32_t dist_bytes, const int32_t *d_cand, int64_t count, int64_t *d_gain,
                  hipStream_t stream);

/*
 * gc_update_dist -- add `node` to S: d(S,.) <- min(d(S,.), d(node,.))
 * (Algorithm "mem-greedy", the update after each pick).  Done by BFS from
 * node pruned to nodes w with d(node,w) < d(S,w), which leaves every other
 * entry unchanged (Section 4.1).
 *   d_dist      device uint8/uint16[n], in/out: d(S,.) -> d(S u {node},.);
 *               all-INF means S = {} (then a full BFS is run)
 *   dist_bytes  1 or 2 (GC_EINVAL otherwise); 4 on a weighted graph
 *   d_farness   device int64, in/out: F(S) -> F(S u {node}); its input is
 *               ignored when S = {}
 * Synchronises the stream every few levels (the depth is found as it goes).
 * Errors: GC_EINVAL for node out of range; GC_ERANGE is reported by a later
 * synchronising call if a distance reached INF (use dist_bytes = 2, or
 * gc_greedy_group, which picks the width itself).
 */
int gc_update_dist(const gc_graph *g, int32_t node, void *d_dist, int32_t dist_bytes, void *d_ws,
                   size_t ws_bytes, hipStream_t stream, int64_t *d_farness);

/*
 * gc_marginal_gains -- g(v,S) = F(S) - F(S u {v}) for count candidates
 * (Section 4.1, pruned SSSP; the per-level counting view is the theorem of
 * Section 4.3).  Candidates are processed in groups of bitset_width sources
 * that share one bit-parallel BFS frontier.  A candidate already in S gets 0.
 * Requires S != {} (d_dist finite everywhere).
 *   d_dist      device uint8/uint16[n] = d(S,.) (int32[n], dist_bytes = 4,
 *               on a weighted graph: one search per candidate, asynchronous)
 *   d_cand      device int32[count], ids in [0,n) (duplicates allowed)
 *   d_gain      device int64[count] out
 *   d_edges     device int64[count] out or NULL: sum_{w in V(v)} deg(w)
 *   d_visited   device int32[count] out or NULL: |V(v)|
 * Synchronises the stream twice: to read max d(S,.) (the BFS depth) and to
 * check the frontier log (an overflowed launch is redone with fewer sources
 * per launch; the results are the same).  An id outside [0, n) touches no
 * memory and gets gain 0 (the Python binding rejects such ids instead).
 */
int gc_marginal_gains(const gc_graph *g, const void *d_dist, int32_t dist_bytes,
                      const int32_t *d_cand, int32_t count, int64_t *d_gain, int64_t *d_edges,
                      int32_t *d_visited, void *d_ws, size_t ws_bytes, hipStream_t stream);

/*
 * gc_marginal_gains_noalloc -- for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same gains as gc_marginal_gains, with every device
 * scratch buffer taken from one array of GC_NOALLOC_SCRATCH_BYTES bytes that
 * the library holds on each GPU it runs on until the process ends.  No
 * workspace argument and no allocation of any kind; the caller passes only
 * inputs and outputs, laid out as for gc_marginal_gains.
 *   Size limit: the graph's split rows (4 nnz bytes), per-node tables (18 n
 *   bytes), frontier ring and clean-up list (28 bytes per entry, n + 128
 *   entries rounded up to a power of two), the level records (1 MiB) and at
 *   least one batch of per-node records (32 n bytes) must fit; otherwise
 *   GC_EWORKSPACE with the bytes needed, and nothing is run.
 *   Every call on one GPU uses the same array and first clears what it reads
 *   before writing, so calls run one after another on that GPU may use
 *   different graphs; calls that overlap in time on one GPU (two streams,
 *   two host threads) race and give undefined results.
 * Synchronises the stream as gc_marginal_gains does.
 */
#define GC_NOALLOC_SCRATCH_BYTES (256u << 20)
int gc_marginal_gains_noalloc(const gc_graph *g, const void *d_dist, int32_t dist_bytes,
                              const int32_t *d_cand, int32_t count, int64_t *d_gain, int64_t *d_edges,
                              int32_t *d_visited, hipStream_t stream);

/*
 * gc_gain_words -- word-level work of the last gc_marginal_gains call on this
 * workspace (the bit-parallel form of Section 4.3: one frontier entry carries
 * every source of a batch that reached a node at the same level).
 *   h_words  host int64[6] out: frontier entries of all levels, of level 0
 *            (roots), of the last level (logged, not expanded); adjacency
 *            entries expanded; adjacency entries of the last level; (batch,
 *            node) records touched (claimed at least once).
 * A frontier entry is a node with neighbours that can still be claimed; its
 * adjacency entries are those neighbours only (rows are split by the d(S,.)
 * of the call, so a node at distance L from its sources expands the
 * neighbours z with d(S,z) >= L + 2).  With one candidate per call the
 * records touched equal |V(v)|.  Synchronises the stream.
 */
int gc_gain_words(const gc_graph *g, const void *d_ws, size_t ws_bytes, hipStream_t stream,
                  int64_t *h_words);

/*
 * gc_greedy_group -- Greedy++ (Section 4): k picks, exactly the picks of the
 * plain greedy of Section 3.2 with smallest-id ties, for every candidate order.
 *   k           1 <= k <= n (GC_EINVAL otherwise)
 *   opts        NULL or options (see gc_opts)
 *   h_group     host out int32[k]: picks in order
 *   h_farness   host out int64[k]: F(S_1), ..., F(S_k)
 *   h_stats     host out or NULL
 * Synchronises the stream.  Weighted graphs: plain or CELF order only (no
 * d_bits, early exit, learned order or log: GC_EINVAL); the first gain round
 * evaluates every node in one launch; stats.dist_bytes = 4, ecc_s1 = 0.
 */
int gc_greedy_group(const gc_graph *g, int32_t k, const gc_opts *opts, void *d_ws,
                    size_t ws_bytes, hipStream_t stream, int32_t *h_group, int64_t *h_farness,
                    gc_stats *h_stats);

/*
 * gc_greedy_many -- gc_greedy_group for `count` independent jobs (graph
 * graphs[i], k[i]) run by `nworkers` host threads.  Worker w works on its own
 * stream streams[w] with its own workspace d_ws[w] of ws_bytes[w] bytes (at
 * least gc_workspace_size of every graph), which it prepares for each job as
 * gc_workspace_init would (the first job on it: gc_workspace_init itself;
 * later jobs: only what the previous job may have left non-zero, since the
 * engine returns every record it touches to zero); jobs go to the next free
 * worker, largest graph first, so independent jobs overlap their launch
 * latencies on the GPU.
 * Every job gets the same picks as gc_greedy_group would give it alone.
 *   count       >= 0 jobs; graphs[i] and k[i] as for gc_greedy_group
 *   opts        NULL or one gc_opts for every job (nprefix must be 0, no log)
 *   nworkers    1..64; streams must not be the null stream when nworkers > 1
 *   h_group     host out int32[sum k]: job i's picks from offset k[0]+..+k[i-1]
 *   h_farness   host out int64[sum k], same offsets
 *   h_stats     NULL or host out gc_stats[count] (h_evals_per_round ignored)
 * Returns when every job has ended: GC_OK, or the error of the lowest-numbered
 * failed job (gc_last_error names it); the other jobs still run.  The graphs
 * are only read; the workspaces and streams must not be used concurrently
 * by anything else.
 */
int gc_greedy_many(int32_t count, const gc_graph *const *graphs, const int32_t *k,
                   const gc_opts *opts, int32_t nworkers, void *const *d_ws, const size_t *ws_bytes,
                   const hipStream_t *streams, int32_t *h_group, int64_t *h_farness,
                   gc_stats *h_stats);

/*
 * gc_greedy_batch -- the jobs of gc_greedy_many (same arguments and the same
 * picks, farness and evaluation counts) with their later rounds run in
 * lockstep.  Phase 1, on the nworkers host threads as in gc_greedy_many:
 * each job's first pick, its first gain round (every candidate) and its
 * second pick.  Phase 2, on streams[0]: every job's later rounds at once --
 * each step, every job still selecting takes its next batch of candidates
 * by the lazy rule of Section 4.2 and one gain call over the disjoint union
 * of all the graphs evaluates them all; the jobs whose round ended get their
 * d(S,.) update in one call.  A batch of 64 sources holds one job's
 * candidates and gets records for that job's nodes only.
 *   d_union, union_bytes  device buffer of at least gc_batch_union_size bytes
 *               (256-byte aligned; the union CSR, its d(S,.) and the engine's
 *               scratch), prepared by the call itself
 *   opts        NULL or plain/CELF order with block and block_growth (no
 *               prefix, log, learned order, bit vectors or early exit)
 *   graphs      unweighted (GC_EINVAL otherwise); the union must have fewer
 *               than 2^31 nodes and adjacency entries (GC_ERANGE)
 *   h_stats     per job: evaluations, E_alg, launches and its phase-1 times;
 *               ms_later is the whole phase 2 and ms_total the whole call
 * Synchronises every stream.  On error the lowest-numbered failed job's
 * error (phase 1) or the call's error (phase 2) is returned.
 */
int gc_batch_union_size(int32_t count, const gc_graph *const *graphs, int32_t block, size_t *bytes);
int gc_greedy_batch(int32_t count, const gc_graph *const *graphs, const int32_t *k, const gc_opts *opts,
                    int32_t nworkers, void *const *d_ws, const size_t *ws_bytes, const hipStream_t *streams,
                    void *d_union, size_t union_bytes, int32_t *h_group, int64_t *h_farness,
                    gc_stats *h_stats);

/* --------------------------------------------- candidate-ordering MLP --- */
/*
 * Not part of the paper's method: a small network that predicts marginal
 * gains so that GC_ORDER_LEARNED evaluates likely winners first.  Exact
 * pruned BFS still decides every pick, so the group and farness do not depend
 * on the network.  8 features -> 64 -> 64 -> 1 with ReLU; weights bfloat16,
 * biases and accumulation float32; target log2(1 + gain).
 *
 * Master parameters: float32[GC_MLP_PARAMS] in the order W1 (64x8, row j =
 * hidden unit j), b1 (64), W2 (64x64, row j = unit j), b2 (64), W3 (64), b3.
 * Inference block: gc_mlp_block_bytes() bytes made by gc_mlp_pack (bf16
 * weights rounded to nearest-even, float32 biases).
 * Rounding points: x = bf16(feature); h1 = bf16(relu(W1 x + b1));
 * h2 = bf16(relu(W2 h1 + b2)); out = W3 h2 + b3 (float32).
 */
#define GC_MLP_INPUTS 8
#define GC_MLP_HIDDEN 64
#define GC_MLP_PARAMS 4801

size_t gc_mlp_block_bytes(void);
/* master float32 -> inference block; asynchronous */
int gc_mlp_pack(const float *d_master, void *d_block, hipStream_t stream);
/*
 * gc_mlp_forward -- out[s] for count samples; d_x float32 [count x 8].
 * d_h1, d_h2: optional float32 [count x 64] activations (as bf16 values),
 * needed by gc_mlp_backward.  Asynchronous.
 */
int gc_mlp_forward(const void *d_block, const float *d_x, int32_t count, float *d_out, float *d_h1,
                   float *d_h2, hipStream_t stream);
/* floats of scratch gc_mlp_backward needs for count samples */
size_t gc_mlp_scratch_floats(int32_t count);
/*
 * gc_mlp_backward -- gradient of the mean squared error
 * (1/count) sum_s (out_s - y_s)^2 with respect to the master parameters,
 * d_grad float32[GC_MLP_PARAMS] in the master layout.  Uses the activations
 * of gc_mlp_forward; products of bf16 values, float32 sums in sample order.
 */
int gc_mlp_backward(const void *d_block, const float *d_x, const float *d_h1, const float *d_h2,
                    const float *d_out, const float *d_y, int32_t count, float *d_grad,
                    float *d_scratch, hipStream_t stream);
/* one Adam step (Kingma and Ba) on the master vector; step counts from 1 */
int gc_mlp_adam(float *d_master, float *d_m, float *d_v, const float *d_grad, int32_t step,
                float lr, float beta1, float beta2, float eps, hipStream_t stream);
/*
 * gc_node_features -- the 8 features of the learned order for count nodes
 * (d_cand, or nodes 0..count-1 when NULL), float32 [count x 8]:
 *   log2(1+deg v), d(S,v)/ecc1, log2(1+ub[v]), log2(1+sum_{u in N(v)} deg u),
 *   log2(1+round-last_eval[v]) (round if never), d_at_eval[v]-d(S,v) (0 if
 *   never), round/k, log2(1+d(S,v)).
 * d_ub int64[n] (stale gains), d_last_eval int32[n] (-1 = never),
 * d_dist_at_eval uint16[n].  Asynchronous.
 */
int gc_node_features(const gc_graph *g, const void *d_dist, int32_t dist_bytes,
                     const int32_t *d_cand, int32_t count, const int64_t *d_ub,
                     const int32_t *d_last_eval, const uint16_t *d_dist_at_eval, int32_t round,
                     int32_t k, int32_t ecc1, float *d_feat, hipStream_t stream);

/* ----------------------------------------------------------------- misc --- */

const char *gc_strerror(int code);
const char *gc_last_error(void);

/*
 * Kernel timing for measurement: with gc_timing_enable(1) every marginal-gain
 * evaluation records two HIP events on its stream, immediately before its
 * first and after its last kernel; gc_timing_last_ms() returns the elapsed
 * time of the last one (-1 if none).  Per host thread.
 */
int gc_timing_enable(int on);
double gc_timing_last_ms(void);

#ifdef __cplusplus
}
#endif
#endif /* GC_H */
