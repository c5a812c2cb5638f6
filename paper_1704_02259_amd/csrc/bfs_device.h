// Shared layout between the host runtime and the gfx950 kernels of libhybfs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hybfs {

constexpr int kBlock = 256;                    // threads per block of the layer kernels
constexpr int kWave = 64;                      // CDNA wavefront
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kFinishBlock = 1024;             // one-block kernels
constexpr int kFinisherBlock = 512;            // the traversal's finisher
constexpr int kSlots = 4;                      // ring of per-layer counter slots

enum { DIR_TD = 0, DIR_BU = 1 };
enum { RULE_EDGES = 0, RULE_TABLE = 1, RULE_TOPDOWN = 2, RULE_BOTTOMUP = 3 };

// Counters of one frontier F_d, accumulated while F_{d-1} is processed.  Each
// block adds into sub-counter blockIdx % kSub, one 64-byte line apart, so the
// atomics of a layer spread over kSub addresses; readers sum the sub-counters.
constexpr int kSub = 16;
struct Slot {
    unsigned long long c[kSub][8];   // c[k][0]: part of |F_d|, c[k][1]: part of sum deg(F_d),
                                     // c[k][2]: part of the count of F_d's vertices above
                                     // hub_deg; c[0][3]: entries of F_d's hub list,
                                     // c[0][4]: entries of F_d's queue (appended by atomics
                                     // on these single addresses)
};
constexpr int kHubTail = 3;
constexpr int kQueueTail = 4;

// How the frontier F_d is available besides its bitmap (LayerState::qform).
enum { QF_NONE = 0,                  // bitmap only
       QF_LIST = 1,                  // queue of F_d; F_d is not yet in vis
       QF_LIST_VIS = 2 };            // queue of F_d; F_d is already in vis

// What the kernel of layer d needs from the layers before it.  Two copies
// alternate: the kernel of layer d reads st[d & 1] and its block 0 writes
// st[(d + 1) & 1], which no block of the same kernel reads.
struct LayerState {
    int d;                           // layer index
    int dir_prev;                    // direction of layer d-1 (top-down before layer 0)
    long long m_u;                   // edges of vertices not in layers 0..d-1
    long long v_u;                   // vertices not in layers 0..d-1
    long long reached;               // vertices in layers 0..d-1
    long long reached_deg;           // their degree sum
    int qform;                       // QF_*: F_d's queue, written by the layer before
    int hlist;                       // 1: F_d's hub list was written (complete unless too long)
    int filt;                        // 1: F_d's membership filter was written
    int pad1;
    long long pad[1];
};

// Trace of one processed layer, written by block 0.
struct LayerRec {
    int dir;
    int pad;
    long long n_f, m_f, m_u, v_u;
};

struct Ctrl {
    int done;                        // set once a layer finds an empty frontier
    int nlayers;
    int parity;                      // which LayerState the next layer reads
    int root;
    long long reached;
    long long reached_deg;
    int *level;                      // outputs of the current traversal
    int *parent;
    int status;                      // nonzero: a device-side consistency check failed
    int bin_layer;                   // layer whose top-down step runs binned, else -1
    int bin_qlen;                    // that layer's frontier: queue length, or -1 for the bitmap
    int bin_hlist;                   // that layer's hubs come from the hub list
    int async_run;                   // the current traversal was enqueued asynchronously
    int fail_injected;               // test hook: the finisher reports a failure (bit 0x200)
    // failures of asynchronous traversals since the host last read them: the
    // finisher of a failed async run adds one to err_runs and ORs its status
    // (and 0x100 when it did not end normally) into err_bits
    unsigned err_runs;
    unsigned err_bits;
    LayerState st[2];
    Slot slot[kSlots];
};

// A top-down work item: the `chunk`-th block of 2^chunk_log2 edges of u.
struct Item {
    int u;
    int chunk;
};

// A segment of a hub row for the batched bottom-up scan: row v, segment
// number seg within the row, and `first`, the index of the row's segment 0
// in the row-major numbering that indexes the found masks.
struct HSeg {
    int v;
    int seg;
    long long first;
};

struct Params {
    long long n, nnz, W;                 // vertices, stored entries, bitmap words
    const long long *off;                // int64 [n+1]
    const int *col;                      // int32 [nnz], rows ascending
    const unsigned long long *iso;       // [W] bit set: degree 0 or v >= n
    const int *deg;                      // int32 [n] row lengths
    const int *slab;                     // int32 [slab_k * n] position-major first
                                         // neighbours: slab[p*n + v] = p-th entry of
                                         // row v, or -1 past its end
    int slab_k;
    int chunk_log2;                      // top-down hub chunks cover 2^chunk_log2 edges
    const Item *hub;                     // every chunk of every vertex of degree > hub_deg
    long long n_hub;
    int hub_deg;                         // top-down cut-off of this run (>= the table's)
    int pad0;
    int probe_k;                         // bottom-up positions tried per lane
    int wpg;                             // bottom-up: bitmap words per wavefront task (1..64)
    int wpg_td;                          // top-down: bitmap words per wavefront task (1..64)
    unsigned long long *vis;             // [W] finished layers (+ iso bits)
    unsigned long long *bm;              // [3W] rotating frontier / next / spare
    int *level, *parent;                 // outputs [n]
    Ctrl *ctrl;
    LayerRec *trace;
    int trace_cap;
    int root;
    int rule;
    long long alpha, beta;
    long long alpha_bin;                 // edge rule's alpha for a layer that would run binned
    int async_run;                       // enqueued asynchronously (failures kept for bfs_graph_sync)
    int first_writer;                    // top-down parents by first writer, not minimum
    // binned top-down (large top-down layers): frontier edges are bucketed by
    // destination tile of 2^bin_log2 vertices, minima taken in LDS per tile
    int *bin_cnt;                        // [nbins] edges per tile (zero between uses)
    int *bin_off;                        // [nbins + 1] bucket offsets
    int *bin_cur;                        // [nbins] bucket fill cursors
    unsigned long long *bin_pairs;       // [bin_cap] (parent << 32 | vertex within tile)
    long long bin_cap;
    long long bin_min_edges;             // smallest m_f that runs binned (when allowed)
    int nbins;
    int bin_log2;
    int serial_probes;                   // bottom-up: test frontier bits one at a time
    int wide;                            // layers run in bfs_layer_kernel_wide
    int fail_injected;                   // test hook: report this traversal as failed
    // frontier queues (Algorithm 1's output queue): q0 (even d) and q1 (odd
    // d) hold F_d as a list of vertex ids, appended by the producers of F_d.
    // Two named pointers, not an array: a runtime index into the parameter
    // block would move the whole block into private memory.
    int *q0, *q1;
    long long q_cap;                     // entries of each (n)
    int td_queue;                        // QM_*: which layers write and read queues
    // hub lists: the 2^chunk_log2-edge chunks of F_d's vertices above hub_deg,
    // appended by whichever step discovers them; a top-down layer expands its
    // hubs from the list instead of scanning the graph's whole hub table
    int hub_list;                        // HL_*: which steps write hub lists
    Item *hq0, *hq1;                     // even and odd layers
    long long hq_cap;                    // entries of each (the table's size bounds them)
    int q_write;                         // set per layer: this layer appends its output to
                                         // the next frontier's queue
    int h_write;                         // set per layer: this layer lists the hubs it discovers
    // membership filters of small frontiers: 2^kFilterLog2 bits (two hashed
    // bits per member), three rotating like the bitmaps; a bottom-up layer
    // whose frontier has one tests it in LDS before each frontier-bit probe
    unsigned *filt;
    int f_write;                         // set per layer: this layer fills the next frontier's filter
    int use_filter;                      // filters are kept and used
    // per-layer work counters (statistics build only): kCounts per layer
    unsigned long long *pstat;
    int count;                           // 1: count (the statistics build runs the layers)
    int pad3;
};

__device__ __forceinline__ int *queue_of(const Params &P, int d) { return (d & 1) ? P.q1 : P.q0; }
__device__ __forceinline__ Item *hubs_of(const Params &P, int d) { return (d & 1) ? P.hq1 : P.hq0; }

// Hub-list modes (Params::hub_list).  A top-down layer reads its frontier's
// hub list whenever the layer before wrote one.
enum { HL_OFF = 0,
       HL_ALL = 1,                       // every step lists the hubs it discovers
       HL_LAYER0 = 2,                    // only layer 0 (the root's row) does, for layer 1
       HL_TD = 3,                        // layer 0 and the top-down steps do
       HL_EARLY = 4 };                   // layer 0 and a top-down layer 1 do, for layers 1 and 2

// Builds of the layer kernel (which lists their code keeps; the last one
// counts the work of each layer instead).
enum { BUILD_PLAIN = 0, BUILD_HUBS = 1, BUILD_QUEUES = 2, BUILD_COUNTS = 3 };

// Work counters of one layer (statistics build).  Bottom-up: vertices
// examined, phase-1 frontier probes, rows continued in phase 2, phase-2
// wavefront steps, phase-2 entries probed, vertices found.  Top-down: edges
// examined, candidates (target in no finished layer), atomic minima issued,
// vertices discovered, and two unused.
constexpr int kCounts = 6;
struct WorkCount {
    unsigned long long c[kCounts];
};

// Queue modes (Params::td_queue).
enum { QM_OFF = 0,                       // bitmaps only
       QM_TOPDOWN = 1,                   // top-down layers (and layer 0) write their output
                                         // queue; a top-down layer reads its input queue
                                         // when the layer before left one
       QM_ALL = 2 };                     // every layer writes its output as a queue too
                                         // (bottom-up and binned steps convert their output
                                         // bitmap words), every top-down layer reads one

constexpr int kFilterLog2 = 17;                // 16 KiB of filter bits, the size of the LDS tile histogram
constexpr int kFilterWords = (1 << kFilterLog2) / 32;
// a top-down layer of at most this many frontier edges fills the filter of its
// output, and a bottom-up layer of at most this many frontier vertices uses it
constexpr long long kFilterMaxEdges = 1 << 16;
constexpr long long kFilterMaxFrontier = 1 << 16;
constexpr int kBinLog2 = 14;                   // destination tile: 16384 vertices, 64 KiB of minima in LDS
constexpr int kMaxBins = 4096;
static_assert(kFilterWords <= kMaxBins, "the LDS filter shares the tile histogram's space");
constexpr int kWideWavesPerSimd = 6;           // residency the wide layer kernel is built for

// ---------------------------------------------------------------------------
// Batched multi-source traversal: lane b of every uint64 mask is root b.
constexpr int kLanes = 64;

// Counters of one batched frontier F_d (per sub-counter line):
//   c[k][0] (root, vertex) pairs in F_d          c[k][1] vertices in any lane's F_d
//   c[k][2] degree sum of those vertices         c[k][3] degree sum of vertices that
//   c[k][4] of them above hub_deg                        became visited in every lane
//   c[k][5] degree sum over the pairs
struct BSlot {
    unsigned long long c[kSub][8];
};

struct BLayerState {
    int d;
    int dir_prev;
    long long m_u;                   // degree sum of vertices not visited in every lane
    long long pairs;                 // (root, vertex) pairs in layers 0..d-1
    long long pairs_deg;             // their degree sum
    long long pad[4];
};

struct BCtrl {
    int done;
    int nlayers;
    int parity;
    int status;
    int async_run;                   // as in Ctrl
    int fail_injected;
    unsigned err_runs;
    unsigned err_bits;
    long long pairs;
    long long pairs_deg;
    long long pad[4];
    BLayerState st[2];
    BSlot slot[kSlots];
};

struct RootSet {
    int r[kLanes];
};

// Output arrays of each lane: level_b[n] and parent_b[n] of root b.
struct LanePtrs {
    int *level[kLanes];
    int *parent[kLanes];
};

struct BParams {
    long long n, nnz, W;
    const long long *off;
    const int *col;
    const int *deg;
    const unsigned long long *iso;
    const Item *hub;
    long long n_hub;
    int hub_log2;
    int hub_deg;
    // bottom-up scans of hub rows: segments of 2^seg_log2 consecutive chunks,
    // listed by segment number (every row's segment 0, then segment 1, ...);
    // sfound holds per segment, numbered row-major, the lanes it has found
    // (cleared per batch)
    const HSeg *hseg;
    long long n_hseg;
    unsigned long long *sfound;
    int seg_log2;
    int k;                               // lanes in use (1..64)
    int rule;
    unsigned long long active;           // bit b set for b < k
    unsigned long long *vis;             // [n] lanes that reached v in a finished layer
    // [(hist + 3) n] lane masks of the layers' frontiers: F_d in slot d for
    // d < hist (kept for the level pass, which clears them), later layers in
    // the three slots after those, rotating (frontier / next / spare)
    unsigned long long *fm;
    unsigned long long *ubm;             // [3W] rotating bitmaps: vertex has a nonzero mask
    int *const *lvl;                     // device table [kLanes]: lane b's level array
    int *const *par;                     // device table [kLanes]: lane b's parent array
    BCtrl *ctrl;
    LayerRec *trace;
    int trace_cap;
    int wpg;                             // pull: bitmap words per wavefront task
    int wpg_td;                          // push: bitmap words per wavefront task
    int async_run;                       // enqueued asynchronously
    long long alpha, beta;
    int fail_injected;                   // test hook: report this batch as failed
    int hist;                            // levels below this come from the kept masks (level pass)
};

// The init kernel copies `out` into the device tables p.lvl / p.par.
hipError_t launch_batch_init(const BParams &p, const LanePtrs &out, int grid, hipStream_t s);
hipError_t launch_batch_seed(const BParams &p, const RootSet &roots, hipStream_t s);
hipError_t launch_batch_push(const BParams &p, int layer, int grid, hipStream_t s);
hipError_t launch_batch_pull(const BParams &p, int layer, int grid, hipStream_t s);   // blocks of kPullWaves waves
hipError_t launch_batch_finish(const BParams &p, hipStream_t s);
hipError_t launch_batch_levels(const BParams &p, int grid, hipStream_t s);
int batch_blocks_per_cu();
int batch_pull_blocks_per_cu();
constexpr int kPullWaves = 4;             // wavefronts per block of the batched pull kernel
// Layers whose frontier masks a batch keeps, so that their levels are stored
// once, after the traversal, instead of by the layers (levels below 16:
// four bit-slices).
constexpr int kBatchHist = 12;
static_assert(kBatchHist >= 1 && kBatchHist <= 16, "kept layers: level 0 always, four bit-slices");

// Launchers (defined in bfs_kernels.hip).
hipError_t launch_init(const Params &p, int grid, hipStream_t s);
// allow_binned: the three binned kernels follow this layer kernel in the stream
hipError_t launch_layer(const Params &p, int layer, int allow_binned, int grid, hipStream_t s);
// the build (BUILD_*) that runs layer `layer`, and the finisher's
int layer_build(const Params &p, int layer);
int finish_build(const Params &p);
hipError_t launch_bin_scan(const Params &p, int layer, hipStream_t s);
hipError_t launch_bin_scatter(const Params &p, int layer, int grid, hipStream_t s);
hipError_t launch_bin_reduce(const Params &p, int layer, int grid, hipStream_t s);
hipError_t launch_finish(const Params &p, hipStream_t s);
// layer 0 in one block (roots of small degree; see kRootKernelDegree)
hipError_t launch_root(const Params &p, hipStream_t s);
constexpr long long kRootKernelDegree = 4096;
// initialisation and layer 0 in one grid-wide kernel: block b owns `per`
// bitmap words (at most kFuseWords); needs every counter slot at zero
hipError_t launch_init_root(const Params &p, int grid, int per, hipStream_t s);
constexpr int kFuseWords = 1024;
hipError_t launch_iso_template(const long long *off, long long n, long long W,
                               unsigned long long *iso, hipStream_t s);
void *kernel_ptr_init();
void *kernel_ptr_layer(bool wide, int build, bool filter);
// whether layer `layer` runs in the wide build with the small-frontier filters
bool layer_filter(const Params &p, int layer);
void *kernel_ptr_finish(int build);
void *kernel_ptr_init_root();
void *kernel_ptr_bin_scan();
void *kernel_ptr_bin_scatter();
void *kernel_ptr_bin_reduce();
// The batched kernels, for graph nodes (arguments as their launchers pass them).
enum { BK_INIT, BK_SEED, BK_PUSH, BK_PULL, BK_FINISH, BK_LEVELS };
void *kernel_ptr_batch(int which);
constexpr int kReduceBlockThreads = 512;   // threads of a binned reduce block
int layer_blocks_per_cu(bool wide);

}  // namespace hybfs
