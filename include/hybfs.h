/*
 * hybfs -- hybrid (direction-optimising) breadth-first search on one MI355X.
 *
 * C ABI of libhybfs.so.  Plain pointers and sizes only.  Every call returns
 * BFS_OK (0) or a negative BFS_E_* code; on error the outputs are unspecified
 * and bfs_last_error() holds a message for the calling thread.  Nothing aborts
 * the process and no C++ exception crosses this boundary.
 *
 * The method (paper Sections 4-5): a layer-synchronous BFS in which each layer
 * is processed either top-down (Algorithm 1: the frontier's adjacency lists
 * are expanded into the output queue) or bottom-up (Algorithm 2: every
 * unvisited vertex scans its adjacency list for a frontier vertex and stops at
 * the first one; Algorithms 4-5 try the first MAX_POS positions of many
 * vertices at once before a plain scan).  An online rule on the frontier size
 * and edge counts (Algorithm 3, Table 2) picks the direction of each layer.
 *
 * Result convention (for every entry point):
 *   level[v]  = hop distance from the root, -1 if v is not reachable;
 *   parent[v] = the smallest-id neighbour of v one layer closer to the root,
 *               parent[root] = root, -1 if v is not reachable.
 * Fixing the tree this way removes the run-to-run freedom a parallel BFS has
 * (Section 7.1), so the output does not depend on the direction schedule,
 * the tuning parameters, batching or concurrency.
 *
 * Graph requirements: n in [1, 2^31-1]; row_offsets[0] = 0, non-decreasing,
 * row_offsets[n] = nnz; col_indices in [0, n).  The graph must be undirected
 * (both directions stored), because the bottom-up step finds a vertex's
 * parents among its own neighbours (Section 4).  Each row must be sorted
 * ascending unless BFS_GRAPH_SORT_ROWS is given.  Self-loops and duplicate
 * entries are allowed and do not change the result.
 */
#ifndef HYBFS_H
#define HYBFS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define BFS_OK           0
#define BFS_E_INVALID   (-1)  /* bad argument or malformed graph */
#define BFS_E_NOMEM     (-2)  /* device or host allocation failed / over budget */
#define BFS_E_DEVICE    (-3)  /* HIP runtime error or device-side failure */
#define BFS_E_BUSY      (-4)  /* queue full (serving) */
#define BFS_E_NOTFOUND  (-5)  /* unknown graph id or ticket */
#define BFS_E_TIMEOUT   (-6)  /* a wait timed out */
#define BFS_E_IO        (-7)  /* a file could not be read or written */

typedef struct bfs_graph *bfs_graph_t;

/* ---- graph creation flags ---- */
#define BFS_GRAPH_DEVICE_INPUT   1u  /* row_offsets / col_indices are device pointers */
#define BFS_GRAPH_ASSUME_VALID   2u  /* skip the host-side structural checks */
#define BFS_GRAPH_CHECK_SYMMETRY 4u  /* also verify that every edge is stored both ways
                                        (runs the structural checks too, even with
                                        BFS_GRAPH_ASSUME_VALID) */
#define BFS_GRAPH_SORT_ROWS      8u  /* rows may be unsorted: sort the library's copy */

/*
 * Make a graph resident on the current HIP device.
 *   n, nnz       vertex count and number of stored (directed) CSR entries.
 *   row_offsets  int64[n+1]; col_indices int32[nnz]; host pointers unless
 *                BFS_GRAPH_DEVICE_INPUT.  The library copies both; the caller
 *                keeps ownership and may free them after the call returns.
 *   flags        BFS_GRAPH_* bits.
 *   out          receives the handle (immutable; safe to share across threads).
 * Besides the copy, the library precomputes per-vertex data used by every
 * traversal: the degree array, the isolated-vertex bitmap, and a
 * position-major copy of the first entries of every row (the vector-friendly
 * layout of Section 5's bottom-up probes).
 * Errors: BFS_E_INVALID (n or nnz out of range, offsets not monotone or not
 * ending at nnz, a column out of range, an unsorted row without
 * BFS_GRAPH_SORT_ROWS, asymmetry when checked), BFS_E_NOMEM, BFS_E_DEVICE.
 */
int bfs_graph_create(int64_t n, int64_t nnz, const int64_t *row_offsets,
                     const int32_t *col_indices, uint32_t flags, bfs_graph_t *out);

/* Free the device copy and all workspaces (waits for the device first).  The
 * caller must not use the handle afterwards, nor destroy a graph that a
 * server still holds.  Errors: BFS_E_INVALID (NULL handle). */
int bfs_graph_destroy(bfs_graph_t g);

typedef struct bfs_graph_info {
    int64_t n;
    int64_t nnz;
    int64_t isolated;        /* vertices of degree 0 */
    int64_t max_degree;
    int64_t device_bytes;    /* graph-resident bytes (CSR + per-vertex data) */
    int64_t workspace_bytes; /* device bytes of one single-root workspace */
    int32_t grid_blocks;     /* default blocks of a layer kernel */
    int32_t block_threads;   /* threads per block of a layer kernel */
    int32_t slab_k;          /* first entries of each row kept position-major for the
                                bottom-up probes */
    int32_t chunk_edges;     /* top-down hub chunk size in edges */
    int32_t typical_layers;  /* layers the adaptive launch currently enqueues */
    int32_t hub_degree;      /* top-down: vertices above this degree are expanded
                                through a grid-wide table of edge chunks */
    int64_t hub_chunks;      /* entries of that table */
    int64_t batch_workspace_bytes; /* device bytes of one batched workspace
                                      (bfs_run_batch), excluding host-output
                                      staging */
    int32_t layer_kernel_wide; /* 1: the layers run in the build of the layer
                                  kernel for more resident wavefronts
                                  (bfs_layer_kernel_wide, graphs of 2^24
                                  vertices and more), 0: bfs_layer_kernel */
    int32_t reserved;
} bfs_graph_info;

/* Sizes and layout parameters of a resident graph, written to the caller's
 * *info.  Errors: BFS_E_INVALID (NULL argument). */
int bfs_graph_info_get(bfs_graph_t g, bfs_graph_info *info);

/* ---- direction rules (Algorithm 3, switch functions f and g) ----
 * BFS_RULE_EDGES : top-down -> bottom-up when m_f * alpha > m_u; bottom-up ->
 *                  top-down when n_f * beta < n (frontier vertices n_f,
 *                  frontier edges m_f, edges of unvisited vertices m_u).
 * BFS_RULE_TABLE : the reading that reproduces Table 2: f = floor(v_u/1024),
 *                  g = floor(n/64), with v_u the unvisited vertex count;
 *                  top-down -> bottom-up when n_f > f, back when n_f < g.
 * BFS_RULE_TOPDOWN / BFS_RULE_BOTTOMUP force one direction on every layer.
 * Either rule starts top-down and is evaluated before every layer. */
#define BFS_RULE_EDGES     0
#define BFS_RULE_TABLE     1
#define BFS_RULE_TOPDOWN   2
#define BFS_RULE_BOTTOMUP  3

typedef struct bfs_options {
    int32_t rule;              /* BFS_RULE_* */
    int32_t alpha;             /* edge rule parameter, > 0 */
    int32_t beta;              /* edge rule parameter, > 0 */
    int32_t probe_k;           /* bottom-up positions tried per vertex before the
                                  wavefront-cooperative scan (MAX_POS of Section
                                  5.2), 0..64 */
    int32_t td_hub_degree;     /* top-down degree cut-off, 256..2^24 (default 256):
                                  a frontier vertex of higher degree is expanded
                                  through the grid-wide table of its 256-edge
                                  chunks, one of lower degree together with its
                                  wavefront's other frontier vertices */
    int32_t grid_blocks;       /* blocks of each layer kernel; 0 = library default */
    int32_t words_per_wave;    /* bitmap words (64 vertices each) one wavefront
                                  task covers: 1, 2, 4, .., 64; 0 = sized from n */
    int32_t layers_per_launch; /* layer kernels enqueued before the single-block
                                  finisher; 0 = adaptive per graph */
    int32_t out_on_device;     /* 1: level_out / parent_out are device pointers */
    int32_t async;             /* 1: return once enqueued (device outputs only, no
                                  stats); device-side failures are recorded and
                                  reported by the next bfs_graph_sync of the graph
                                  on the same stream */
    int32_t profile_layers;    /* 1: bracket every layer kernel with HIP events on
                                  the stream and report their durations in stats
                                  (synchronous runs with stats only) */
    int32_t graph_launch;      /* 1: replay a hipGraph of the launch sequence,
                                  captured once per workspace and option set, with
                                  only the root(s) and the output pointers updated
                                  per run (bfs_run: one traversal; bfs_run_batch:
                                  each group of up to 64 roots); runs with
                                  profile_layers launch directly (the per-layer
                                  events sit between the launches); 0 (default):
                                  enqueue the kernels one by one (measured as fast
                                  on MI355X for these sequences) */
    int32_t td_binned;         /* large top-down layers bucketed by destination tile
                                  (parents by LDS minimum, outputs written tile by
                                  tile): 0 (default) = for graphs of at least 2^23
                                  vertices, on layers 1..5 with at least 2^22
                                  frontier edges; 1 = every top-down layer; -1 = never */
    int32_t first_writer;      /* 1: top-down parents are first-writer-wins (the
                                  edge that sets a vertex's next-frontier bit
                                  writes its parent, as Algorithm 1 does): levels
                                  are unchanged, parents are some neighbour one
                                  layer closer, no longer the smallest.  Measures
                                  what canonical parents cost; single-root runs
                                  only (batches stay canonical).  0 (default):
                                  canonical parents */
    int32_t bu_serial_probes;  /* bottom-up phase 1 tests the frontier bits of a
                                  vertex's leading neighbours one at a time and
                                  stops at the first hit (1), or all at once to
                                  overlap their latency (-1); 0 (default): one at
                                  a time when the frontier bitmap is 2 MiB or more
                                  (n >= 2^24), where each probe costs a cache line
                                  of bandwidth */
    int32_t td_queue;          /* frontier queues (Algorithm 1's output queue, with
                                  the bitmap/queue conversions of Section 4): a
                                  top-down layer whose frontier was also written as
                                  a queue expands the queue instead of scanning the
                                  frontier bitmap.  1 = top-down layers (and layer 0)
                                  append what they discover to the next queue
                                  (wavefront-aggregated appends) and a top-down layer
                                  after one of them reads it; 2 = every layer writes
                                  its output as a queue too (bottom-up and binned
                                  steps convert their output bitmap words), so every
                                  top-down layer reads one; -1 = bitmaps only;
                                  0 (default) = the library's choice */
    void   *stream;            /* hipStream_t to run on; NULL = default stream */
    int32_t td_hub_list;       /* hub lists: a step that discovers a vertex above
                                  the top-down degree cut-off appends its edge
                                  chunks to the next frontier's hub list, and a
                                  top-down layer whose frontier has such a list
                                  expands its hubs from it instead of scanning the
                                  graph's whole table of hub chunks against the
                                  frontier bitmap (a list longer than a quarter of
                                  the table is abandoned for the table).  1 = every
                                  step keeps them; 2 = only layer 0 (the root's
                                  row), for layer 1; 3 = layer 0 and the top-down
                                  steps; 4 = layer 0 and a top-down layer 1, for
                                  layers 1 and 2; -1 = never; 0 (default) = the
                                  library's choice (2 on graphs of 2^24 vertices and
                                  more, else -1) */
    int32_t alpha_binned;      /* edge rule for a layer whose top-down step would run
                                  binned (td_binned): stay top-down while
                                  m_f * alpha_binned <= m_u, even where alpha says
                                  bottom-up.  The binned step streams its edges
                                  instead of issuing a random atomic per edge, so
                                  its switch point is its own (Algorithm 3's f is
                                  architecture specific).  0 (default) = the
                                  library's choice (alpha where no layer bins) */
    int32_t bu_filter;         /* membership filter of small frontiers: a top-down
                                  layer of at most 2^16 frontier edges sets two
                                  hashed bits per discovered vertex in a 2^17-bit
                                  filter, and a following bottom-up layer of at most
                                  2^16 frontier vertices loads it into LDS and tests
                                  it before each frontier-bit probe (most probes of
                                  such a layer miss, and the filter answers them
                                  without the frontier bitmap).  Only on graphs that
                                  run the wide build of the layer kernel (2^24
                                  vertices and more).  1 = on, -1 = off, 0 (default)
                                  = the library's choice */
    int32_t count_work;        /* 1: count each layer's work on the device and report
                                  it in stats->layers[i].work (synchronous runs with
                                  stats only).  The layers then run in a build of the
                                  layer kernel that counts (slower; frontier queues
                                  off); results are unchanged.  0 (default): no counts */
} bfs_options;

/* Fill defaults: edge rule, alpha 14, beta 24, probe_k 8, td_hub_degree 256,
 * automatic grid / words_per_wave / layers_per_launch, host outputs,
 * synchronous, NULL stream. */
void bfs_options_init(bfs_options *opt);

/* One processed layer d (frontier F_d = vertices at level d). */
typedef struct bfs_layer_stat {
    int32_t direction;  /* 0 top-down, 1 bottom-up */
    int32_t reserved;
    int64_t n_f;        /* |F_d| */
    int64_t m_f;        /* sum of degrees over F_d */
    int64_t m_u;        /* sum of degrees over vertices not in layers 0..d */
    int64_t v_u;        /* number of vertices not in layers 0..d */
    double  t_us;       /* time of this layer (HIP events, profile_layers runs
                           only, else 0); layers past the enqueued kernels,
                           run by the finisher, report 0 */
    double  kernel_us;  /* HIP-event duration of this layer's kernel (profile_layers), else 0 */
    int64_t work[6];    /* count_work runs only, else 0.  Bottom-up layer: vertices
                           examined, phase-1 frontier probes (the first probe_k
                           positions of each row, Algorithms 4-5), rows continued in
                           phase 2 (the wavefront-cooperative scan of Algorithm 2),
                           phase-2 wavefront steps of 64 entries, phase-2 entries
                           probed, vertices found.  Top-down layer (Algorithm 1):
                           edges examined, candidate targets (in no finished layer),
                           atomic updates issued, vertices discovered, 0, 0.  A
                           binned top-down layer reports 0 */
} bfs_layer_stat;

typedef struct bfs_stats {
    int32_t capacity;        /* in: entries available in `layers` (may be 0) */
    int32_t num_layers;      /* out: layers processed (deepest level + 1) */
    bfs_layer_stat *layers;  /* in: caller-owned array of `capacity`, or NULL */
    int64_t reached;         /* out: vertices with level >= 0 */
    int64_t reached_degree_sum; /* out: stored entries of reached vertices;
                                   half of it is the TEPS numerator (Section 6.3) */
    double  device_us;       /* out: HIP-event time of the whole traversal */
    int32_t layer_launches;  /* out: launches of the layer kernel (some may
                                find the traversal already finished); layer 0
                                is not among them when layer0_kernel != 0 */
    int32_t layer0_kernel;   /* out: where layer 0 ran: 0 the layer kernel,
                                1 a one-block kernel, 2 the initialisation
                                kernel (roots of degree <= 4096); batched
                                runs report 0 */
    double  layer_kernel_us; /* out: sum of the HIP-event durations of those
                                layer-kernel launches (profile_layers), else 0 */
} bfs_stats;

/*
 * Single-root hybrid BFS (Algorithm 3 over Algorithms 1 and 2).
 *   root                  vertex id in [0, n).
 *   level_out, parent_out int32[n] each, caller-owned; device pointers if
 *                         opt->out_on_device, else host pointers.
 *   opt                   may be NULL (defaults).
 *   stats                 may be NULL.  Not allowed with opt->async.
 * Enqueued on opt->stream as one init kernel, one kernel per layer (each
 * decides its direction on the device from the frontier counters), and a
 * single-block finisher for layers beyond the enqueued ones.  Concurrent
 * calls on different streams are allowed (each stream gets its own
 * workspace); calls on one stream are ordered by the stream.
 * Errors: BFS_E_INVALID, BFS_E_NOMEM, BFS_E_DEVICE.
 */
int bfs_run(bfs_graph_t g, int32_t root, int32_t *level_out, int32_t *parent_out,
            const bfs_options *opt, bfs_stats *stats);

/*
 * Batched multi-source BFS: k independent single-root traversals sharing one
 * pass over the adjacency lists per layer.  Roots are taken in groups of 64;
 * within a group, bit b of a per-vertex 64-bit mask stands for root b, so the
 * frontier of every root is expanded (Algorithm 1) or probed (Algorithm 2) by
 * one read of each row, and one direction decision (Algorithm 3, edge rule on
 * counts over the union of the roots' frontiers) covers the whole group.  The
 * result for root i is exactly what bfs_run(roots[i]) returns, bit for bit.
 *   roots                 int32[k] host array, each in [0, n); repeats allowed.
 *   k                     >= 1.
 *   level_out, parent_out int32[k * n] each, root-major: root i's arrays start
 *                         at element i * n.  Device pointers if
 *                         opt->out_on_device, else host pointers.
 *   opt                   as for bfs_run, except: rule must be BFS_RULE_EDGES,
 *                         BFS_RULE_TOPDOWN or BFS_RULE_BOTTOMUP; with
 *                         graph_launch each group of up to 64 roots is one
 *                         hipGraph launch (init, seed, the layers' push and
 *                         pull kernels, finisher), captured once per group
 *                         size and option set; probe_k is not used (the pull scans each
 *                         row until every pending root has found a parent).
 *   stats                 may be NULL; not allowed with opt->async.  reached
 *                         and reached_degree_sum are summed over the roots,
 *                         num_layers is the deepest root's, layer_launches
 *                         counts push and pull kernels, device_us sums the
 *                         groups.  `layers` describes the first group: n_f and
 *                         m_f count the union of its roots' frontiers, m_u the
 *                         degree sum of vertices some root has not reached,
 *                         v_u is -1.
 * Errors: BFS_E_INVALID, BFS_E_NOMEM, BFS_E_DEVICE.
 */
int bfs_run_batch(bfs_graph_t g, const int32_t *roots, int32_t k, int32_t *level_out,
                  int32_t *parent_out, const bfs_options *opt, bfs_stats *stats);

/* ---- autotuning ----
 * Coordinate descent over the options that change speed but never results:
 * alpha and beta of the edge rule (Algorithm 3), probe_k (MAX_POS, Section
 * 5.2), td_hub_degree, words_per_wave and grid_blocks; the last four only
 * for single-root mode, alpha/beta/words_per_wave/grid_blocks for batches.
 * Each option set is timed with HIP events on opt->stream: one untimed pass,
 * then the best of two timed passes over the roots (mode 0: bfs_run of each
 * root in turn; mode 1: one bfs_run_batch of all k roots).  A candidate
 * replaces the incumbent only when it is at least 2% faster; descent stops
 * after a round without improvement, four rounds, or max_trials timings.
 *   roots, k     the roots to time (host array, each in [0, n)); tuning on
 *                roots other than those later measured avoids fitting them.
 *   opt          in: starting options (rule, stream, ...); out: the best set
 *                found, with the caller's stream / out_on_device / async /
 *                profile_layers kept.
 *   report       may be NULL.
 * Device scratch for the outputs is allocated and freed inside the call.
 * Errors: BFS_E_INVALID, BFS_E_NOMEM, BFS_E_DEVICE. */
typedef struct bfs_tune_report {
    int32_t trials;          /* option sets timed */
    int32_t rounds;          /* descent rounds */
    double  start_us;        /* time of one pass with the starting options */
    double  best_us;         /* time of one pass with the returned options */
} bfs_tune_report;

int bfs_autotune(bfs_graph_t g, const int32_t *roots, int32_t k, int32_t mode, int32_t max_trials,
                 bfs_options *opt, bfs_tune_report *report);

/* ---- persisted autotune table ----
 * Tuned options outlive the process in a table file: JSON lines, one object
 * per tuned graph, device and mode, with the key fields (and the graph's
 * SCALE = ceil(log2 n) and edgefactor = round(nnz / 2n), for the reader),
 * the tuned options and the tuned time.  MAX_POS (Section 5.2) and the
 * switch parameters of Algorithm 3 are per-graph, per-machine constants,
 * which is what the table keeps. */
typedef struct bfs_tune_key {
    int64_t n, nnz;          /* the graph's vertices and stored entries */
    int64_t max_degree;      /* its largest row */
    int64_t isolated;        /* its vertices without edges */
    int32_t cus;             /* compute units of the device it was tuned on */
    int32_t mode;            /* 0 single-root, 1 batched (as bfs_autotune) */
} bfs_tune_key;

/* The key of graph g on its device for a mode.  Errors: BFS_E_INVALID. */
int bfs_tune_key_get(bfs_graph_t g, int32_t mode, bfs_tune_key *key);

/* Look the key up in the table at `path` (a host file path).  On a hit the
 * tuned fields of *opt (alpha, beta, probe_k, td_hub_degree, grid_blocks,
 * words_per_wave, bu_serial_probes, alpha_binned) are overwritten and the
 * rest kept, and *best_us (may be NULL) receives the stored time; of several
 * entries with the key the last one counts, and lines that do not parse or
 * hold invalid options are skipped.  Errors: BFS_E_NOTFOUND (no such entry,
 * or no such file), BFS_E_INVALID (NULL argument), BFS_E_IO (unreadable). */
int bfs_tune_table_get(const char *path, const bfs_tune_key *key, bfs_options *opt, double *best_us);

/* Record *opt's tuned fields under the key in the table at `path`,
 * replacing any entry with the same key and keeping the others; the file is
 * rewritten through a temporary file in the same directory and renamed, so
 * a reader never sees a partial table.  Calls are serialised, in one
 * process by a mutex and across processes by an exclusive flock() on
 * "<path>.lock" (created beside the table and left there), so concurrent
 * puts of different keys all survive.  Errors: BFS_E_INVALID (NULL argument,
 * invalid options), BFS_E_IO (the file, its temporary or the lock file
 * cannot be written). */
int bfs_tune_table_put(const char *path, const bfs_tune_key *key, const bfs_options *opt, double best_us);

/* ---- serving (continuous batching over resident graphs) ----
 *
 * Not part of the paper: a request layer over bfs_run and bfs_run_batch,
 * which implement its Algorithms 1-3.
 *
 * A server holds graphs that are already resident (bfs_graph_create) and
 * answers single-root BFS queries on them.  `streams` worker slots, each
 * with its own HIP stream and host thread, run traversals concurrently, so
 * the kernels of different queries overlap on the device.  A free slot takes
 * the graph whose oldest queued query has waited longest and drains up to
 * max_batch queued queries of that graph into one traversal: bfs_run for a
 * single query, the batched multi-source traversal (bfs_run_batch) for more
 * (only once enough are queued, see batch_threshold).
 * Queries that arrive while others run wait for the next free slot
 * (continuous batching).  Admission by memory: the slots hold at most
 * memory_budget device bytes.  Charged is everything a slot's traversals
 * leave allocated: the workspaces cached with each graph for the slot's
 * stream (single-root workspace, binned top-down buckets, frontier queues
 * and hub lists, host-output staging; batched workspace) and the slot's
 * host-output staging of batches, plus, while a traversal runs, what it may
 * still allocate.  The graphs' own CSR arrays are not charged.  When a
 * traversal does not fit, idle holdings are released (the slot's own caches
 * of other graphs first, then other idle slots'), then a batch is halved,
 * then the slot waits for running traversals to finish; a query that does not
 * fit with nothing running fails with BFS_E_NOMEM.  Every answer equals
 * bfs_run's for the same graph and root, byte for byte, whatever else is in
 * flight.
 */
typedef struct bfs_server *bfs_server_t;

typedef struct bfs_serve_config {
    int64_t memory_budget;   /* device bytes for traversals in flight; 0 = 75% of the
                                free device memory when the server is created */
    int32_t max_batch;       /* queries per traversal, 1..64 (default 64) */
    int32_t streams;         /* worker slots, 1..16 (default 4) */
    int32_t queue_capacity;  /* queued + running queries before submit returns
                                BFS_E_BUSY, >= 1 (default 65536) */
    int32_t out_on_device;   /* 1 (default): level_out / parent_out of every query are
                                device pointers; 0: host pointers */
    int32_t alpha;           /* switch parameters of Algorithm 3's edge rule, 0 = the */
    int32_t beta;            /* bfs_options defaults */
    int32_t batch_threshold; /* queued queries of one graph from which a slot runs them
                                as one batched traversal; below it a slot takes a
                                single query.  0 (default): adaptive per graph, the
                                ratio of the measured batched and single-root
                                traversal times (2 before anything is measured, 16
                                before a batch is) */
    int32_t reserved;
} bfs_serve_config;

/* Defaults: budget 0 (75% of free memory), max_batch 64, 4 streams, queue
 * capacity 65536, device outputs, default alpha and beta. */
void bfs_serve_config_init(bfs_serve_config *cfg);

typedef struct bfs_serve_report {
    int64_t submitted;       /* since creation or the last bfs_serve_reset_stats */
    int64_t completed;       /* finished with BFS_OK */
    int64_t failed;          /* finished with an error */
    int64_t queued;          /* waiting now */
    int64_t running;         /* in flight now */
    int64_t batches;         /* traversals launched (single or batched) */
    int64_t batched_requests;/* queries answered by a traversal of more than one root */
    int64_t admission_waits; /* times a slot waited for memory to free up */
    int64_t bytes_in_use;    /* device bytes the slots hold or have reserved now */
    int64_t peak_bytes;      /* maximum of bytes_in_use (<= memory_budget) */
    int64_t memory_budget;
    double  p50_us;          /* latency = completion - submission (host monotonic clock), */
    double  p99_us;          /* over completed queries */
    double  mean_us;
    double  max_us;
    double  traversed_edges; /* sum over completed queries of half the reached degree sum */
    double  gteps;           /* traversed_edges / (last completion - first submission) / 1e9 */
    int64_t evictions;       /* idle cached workspaces or staging released for admission */
} bfs_serve_report;

/* Create a server on the current HIP device.  cfg may be NULL (defaults).
 * Errors: BFS_E_INVALID (a field out of range), BFS_E_NOMEM, BFS_E_DEVICE. */
int bfs_serve_create(const bfs_serve_config *cfg, bfs_server_t *out);

/* Register a resident graph; *graph_id receives its id (0, 1, ...).  The
 * caller keeps ownership and must not destroy the graph before the server.
 * Errors: BFS_E_INVALID (NULL argument). */
int bfs_serve_add_graph(bfs_server_t s, bfs_graph_t g, int32_t *graph_id);

/* Queue one BFS query.  level_out / parent_out: int32[n] each, caller-owned,
 * device or host pointers as configured; they must stay valid until the
 * query completes.  *ticket identifies the query.  Errors: BFS_E_NOTFOUND
 * (graph id), BFS_E_INVALID (root out of range, NULL pointer), BFS_E_BUSY
 * (queue_capacity reached). */
int bfs_serve_submit(bfs_server_t s, int32_t graph_id, int32_t root, int32_t *level_out,
                     int32_t *parent_out, uint64_t *ticket);

/* *done = 1 once the query has finished; the call that reports completion
 * releases the ticket and returns the query's own status (BFS_OK or its
 * error).  Unknown or released ticket: BFS_E_NOTFOUND. */
int bfs_serve_poll(bfs_server_t s, uint64_t ticket, int32_t *done);

/* Block until the query finishes (timeout_us < 0: no limit), release the
 * ticket and return the query's status; BFS_E_TIMEOUT leaves it pending. */
int bfs_serve_wait(bfs_server_t s, uint64_t ticket, int64_t timeout_us);

/* Counters and latency percentiles (see bfs_serve_report), written to the
 * caller's *out.  Errors: BFS_E_INVALID (NULL argument). */
int bfs_serve_stats(bfs_server_t s, bfs_serve_report *out);

/* Zero the counters and latencies (e.g. after warm-up queries).
 * Errors: BFS_E_INVALID (NULL server). */
int bfs_serve_reset_stats(bfs_server_t s);

/* Finish every queued and running query, then stop the workers, release the
 * workspaces the server's traversals cached with the graphs, and free the
 * server (graphs are not freed).  Errors: BFS_E_INVALID (NULL server). */
int bfs_serve_destroy(bfs_server_t s);

/* Wait for all work enqueued on `stream` (a HIP stream handle, NULL for the
 * default stream) and report failures of the asynchronous runs of g on that
 * stream (bfs_run and bfs_run_batch with opt->async = 1) since the previous
 * bfs_graph_sync of g on that stream.  The finisher of every traversal
 * records whether it ended normally and passed the device-side consistency
 * checks; this call reads that record and clears it.  Outputs of a failed
 * run are unspecified.
 * Errors: BFS_E_INVALID (NULL graph), BFS_E_DEVICE (a HIP error, or at least
 * one asynchronous run failed: the message counts them and names the status
 * bits). */
int bfs_graph_sync(bfs_graph_t g, void *stream);

/* ---- traversal without device allocation ----
 *
 * For callers that cannot allocate device memory: code that must not call
 * hipMalloc (work recorded under stream capture, tight serving loops, hosts
 * that forbid allocation after start-up).
 *
 * Same traversal and result as bfs_run (byte for byte), but its device scratch
 * (visited bitmap, the three rotating frontier bitmaps, control block and
 * layer trace) lives in one file-scope device array of the library instead
 * of a per-stream workspace.  The array holds graphs of up to
 * BFS_NOALLOC_MAX_VERTICES vertices (32.2 MiB); every device the library is
 * loaded on holds its own copy until the process ends.  The call allocates
 * no device or pinned memory: no hipMalloc, hipFree or allocating library
 * routine.  Differences from bfs_run:
 *   - outputs must be device pointers (opt->out_on_device = 1; with opt ==
 *     NULL the defaults are taken with device outputs);
 *   - synchronous only: opt->async, opt->profile_layers and opt->graph_launch
 *     must be 0;
 *   - the binned top-down step is not used (its buckets would need an
 *     allocation; results do not depend on it);
 *   - stats->device_us, the per-layer times and work counts are 0 (no
 *     events, no count_work).
 * The graph must live on the current device.  All calls on one device share
 * its array, which keeps the last call's contents; the library runs them one
 * at a time (a lock per device), so concurrent calls from several threads
 * queue up rather than race.  The array is initialised on the first call on
 * each device.
 * Errors: BFS_E_INVALID (graph larger than BFS_NOALLOC_MAX_VERTICES, host or
 * asynchronous outputs, graph on another device, bad root or options),
 * BFS_E_DEVICE.
 */
#define BFS_NOALLOC_MAX_VERTICES (1LL << 26)
int bfs_run_noalloc(bfs_graph_t g, int32_t root, int32_t *level_out, int32_t *parent_out,
                    const bfs_options *opt, bfs_stats *stats);

/* Message for the last failed call on this thread ("" if none). */
const char *bfs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HYBFS_H */
