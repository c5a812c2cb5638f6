// Host-side objects behind the opaque handles of include/hybfs.h.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hybfs.h"
#include "bfs_device.h"

namespace hybfs {

constexpr int kTraceCap = 4096;      // per-layer trace records kept on the device
constexpr int kChunkLog2 = 8;        // top-down hub chunks cover 256 edges
constexpr int kSegLog2 = 3;          // batched bottom-up: hub rows in segments of 8 chunks
constexpr int kHubDegree = 256;      // above this degree, rows are split into hub-table chunks
// Default layer-kernel blocks per CU (fewer where the occupancy query allows
// fewer): five 256-thread blocks keep more dependent probe chains in flight
// on the large bottom-up layers than four and cost nothing on small graphs;
// a grid beyond one resident wave of blocks was slower.
constexpr int kLayerBlocksPerCu = 5;
// From this many vertices the layers run in the wide build of the layer
// kernel (six wavefronts per SIMD), six blocks per CU.
constexpr long long kWideMinVertices = 1LL << 24;
constexpr int kWideBlocksPerCu = 6;
// the batched bottom-up keeps a row position below hub_deg in one byte
static_assert(kHubDegree <= 256, "batched pull stages row positions as bytes");

// Per-stream scratch of a single-root traversal.
struct Workspace {
    std::mutex mu;
    void *dbuf = nullptr;
    size_t bytes = 0;
    unsigned long long *vis = nullptr;
    unsigned long long *bm = nullptr;
    Ctrl *ctrl = nullptr;
    LayerRec *trace = nullptr;
    unsigned *filt = nullptr;     // three membership filters of small frontiers
    unsigned long long *pstat = nullptr;   // per-layer work counters (count_work), on first use
    int *out_tmp = nullptr;       // level + parent staging for host outputs
    long long out_tmp_n = 0;
    Ctrl *h_ctrl = nullptr;       // pinned
    LayerRec *h_trace = nullptr;  // pinned
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<hipEvent_t> layer_ev;   // profile_layers: start/end per layer kernel
    // every counter slot of `ctrl` is zero when the stream reaches the next
    // traversal (the workspace was just cleared, or the last traversal was
    // enqueued in full: its finisher clears them)
    bool counters_zero = true;
    // the scratch of bfs_run_noalloc: nothing may be allocated for it
    bool no_alloc = false;
    // binned top-down buckets (allocated on first use)
    void *bin_buf = nullptr;
    int *bin_cnt = nullptr, *bin_off = nullptr, *bin_cur = nullptr;
    unsigned long long *bin_pairs = nullptr;
    long long bin_cap = 0;
    size_t bin_bytes = 0, q_bytes = 0, hq_bytes = 0;
    // frontier queues (2 x n ids) and hub lists (2 x hub-table entries),
    // allocated with the first run that uses them
    void *q_buf = nullptr;
    int *q[2] = {nullptr, nullptr};
    void *hq_buf = nullptr;
    Item *hq[2] = {nullptr, nullptr};
    long long hq_cap = 0;
    // captured launch sequences: key = option set and layer count
    struct Replay {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipGraphNode_t init = nullptr;
        Params params;
        bool fused = false;            // layer 0 runs in the initialisation node
    };
    std::map<std::string, Replay> replays;
    size_t held() const;          // device bytes this workspace holds
    ~Workspace();
};

// Per-stream scratch of a batched traversal (up to 64 roots per group).
struct BatchWorkspace {
    std::mutex mu;
    void *dbuf = nullptr;
    size_t bytes = 0;
    unsigned long long *vis = nullptr;   // [n]
    unsigned long long *fm = nullptr;    // [(kBatchHist + 3) n]: kept, then rotating
    unsigned long long *ubm = nullptr;   // [3W]
    unsigned long long *sfound = nullptr;  // [n_hseg] lanes each hub-row segment found
    BCtrl *ctrl = nullptr;
    LayerRec *trace = nullptr;
    int **tab = nullptr;                 // device [2 * kLanes]: per-lane level, then parent arrays
    int *out_tmp = nullptr;              // host-output staging: level + parent of one group
    long long out_tmp_elems = 0;
    BCtrl *h_ctrl = nullptr;             // pinned
    LayerRec *h_trace = nullptr;         // pinned
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<hipEvent_t> layer_ev;
    // captured launch sequences of one group: key = lanes, option set and
    // layer count; a run rewrites the init node (output table, run flags)
    // and the seed node (roots)
    struct Replay {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipGraphNode_t init = nullptr, seed = nullptr;
        int grid = 0, layers = 0;
    };
    std::map<std::string, Replay> replays;
    size_t held() const { return (dbuf ? bytes : 0) + (out_tmp ? (size_t)out_tmp_elems * 4 : 0); }
    ~BatchWorkspace();
};

// Launch depth of the layered kernels: the deepest of the last 16 traversals,
// clamped to [2, 64].  Deeper traversals are completed by the finisher.
struct DepthTracker {
    std::atomic<int> typical{10};
    std::atomic<int> recent[16];
    std::atomic<unsigned> pos{0};
    DepthTracker()
    {
        for (auto &r : recent) r.store(0);
    }
    void note(int nlayers);
};

struct Graph {
    int dev = 0;
    long long n = 0, nnz = 0, W = 0;
    long long *d_off = nullptr;
    int *d_col = nullptr;
    unsigned long long *d_iso = nullptr;
    int *d_deg = nullptr;
    int *d_slab = nullptr;
    int slab_k = 0;
    Item *d_hub = nullptr;        // top-down chunks of vertices above hub_deg
    long long n_hub = 0;
    HSeg *d_hseg = nullptr;       // batched bottom-up: segments of 2^kSegLog2 chunks of those rows
    long long n_hseg = 0;
    int hub_deg = 0;
    long long isolated = 0, max_degree = 0;
    std::vector<int32_t> h_deg;   // host copy of the degrees (launch choices)
    int cus = 0;
    int blocks_per_cu = 0;
    bool wide = false;                   // layers in the wide build of the layer kernel
    int grid_default = 0;
    int wpg_default = 1;
    DepthTracker depth;                  // single-root traversals
    DepthTracker batch_depth;            // batched traversals
    int nbins = 0;                       // binned top-down: destination tiles
    bool bin_auto = false;               // binned top-down on by default (large graphs)
    int batch_grid = 0;                  // blocks of the batched push kernel
    int batch_pull_grid = 0;             // blocks of the batched pull kernel (kPullWaves waves each)
    int fail_root = -1;                  // test hook (HYBFS_TEST_FAIL_ROOT): traversals from this
                                         // root report a device-side failure
    std::mutex mu;
    std::map<void *, std::unique_ptr<Workspace>> ws;
    std::map<void *, std::unique_ptr<BatchWorkspace>> bws;
};

int set_error(int code, const char *fmt, ...);
void clear_error();
const char *last_error();
int hip_fail(hipError_t e, const char *what);
int validate_options(const bfs_options &o);
int check_csr(int64_t n, int64_t nnz, const int64_t *off, const int32_t *col, bool need_sorted,
              bool check_symmetry);
int get_workspace(Graph *g, void *stream, Workspace **out);
// The queue mode (QM_*) and hub-list flag a run with these options uses.
void queue_modes(const Graph *g, const bfs_options &opt, int *td_queue, int *hub_list);
// Device bytes a workspace adds for the frontier queues and hub lists.
size_t queue_bytes(const Graph *g, bool queues, bool hub_lists);
// Failures of asynchronous traversals of g on `stream` since the last call
// (the stream must be synchronized): BFS_E_DEVICE with a message, and the
// record cleared; BFS_OK when there were none.
int check_async_errors(Graph *g, void *stream);
size_t batch_workspace_bytes(const Graph *g);
// Zeroes `bytes` (a multiple of 8) at p on stream s (bfs_util.hip): a kernel
// rather than a memset, so that a caller capturing the stream records no
// memset node.
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);
// Device bytes the workspaces of g for `stream` hold (single-root and
// batched, each optionally returned), and their release (the stream must be
// idle, the workspaces unused); the device bytes the single-root workspace of
// g on `stream` holds after a bfs_run with these options.
size_t held_bytes(Graph *g, void *stream, size_t *single, size_t *batch);
void release_workspaces(Graph *g, void *stream);
size_t single_run_bytes(Graph *g, void *stream, const bfs_options &opt);
int get_batch_workspace(Graph *g, void *stream, BatchWorkspace **out);
int enqueue_batch(Graph *g, BatchWorkspace *w, const bfs_options &opt, const int32_t *roots, int k,
                  const LanePtrs &out, hipStream_t s, bool profile, int *layers_enqueued);
// The same sequence as one hipGraph launch (captured on first use).
int enqueue_batch_graph(Graph *g, BatchWorkspace *w, const bfs_options &opt, const int32_t *roots, int k,
                        const LanePtrs &out, hipStream_t s, int *layers_enqueued);
void fill_params(const Graph *g, const Workspace *w, const bfs_options &opt, Params *P);
int enqueue_traversal(Graph *g, Workspace *w, const bfs_options &opt, int root, int *lvl, int *par,
                      hipStream_t s, int *layers_enqueued, bool profile, int *layer0_kernel = nullptr);

}  // namespace hybfs
