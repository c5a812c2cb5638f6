// Host runtime and C ABI of libhybfs: graph residency, per-stream workspaces,
// the launch sequence of a traversal, statistics, and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/hybfs.h"
#include "bfs_device.h"
#include "hybfs_internal.h"

namespace hybfs {

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

int set_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

void clear_error() { g_err.clear(); }

const char *last_error() { return g_err.c_str(); }

int hip_fail(hipError_t e, const char *what)
{
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return set_error(BFS_E_NOMEM, "%s: %s", what, hipGetErrorString(e));
    return set_error(BFS_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ------------------------------------------------------------------ CSR checks
int check_csr(int64_t n, int64_t nnz, const int64_t *off, const int32_t *col, bool need_sorted,
              bool check_symmetry)
{
    if (off[0] != 0) return set_error(BFS_E_INVALID, "row_offsets[0] = %lld, expected 0", (long long)off[0]);
    for (int64_t v = 0; v < n; ++v)
        if (off[v + 1] < off[v])
            return set_error(BFS_E_INVALID, "row_offsets decreases at vertex %lld", (long long)v);
    if (off[n] != nnz)
        return set_error(BFS_E_INVALID, "row_offsets[n] = %lld but nnz = %lld", (long long)off[n],
                         (long long)nnz);
    for (int64_t j = 0; j < nnz; ++j)
        if (col[j] < 0 || (int64_t)col[j] >= n)
            return set_error(BFS_E_INVALID, "col_indices[%lld] = %d out of range", (long long)j, col[j]);
    if (need_sorted) {
        for (int64_t v = 0; v < n; ++v)
            for (int64_t j = off[v] + 1; j < off[v + 1]; ++j)
                if (col[j] < col[j - 1])
                    return set_error(BFS_E_INVALID,
                                     "row %lld is not sorted ascending (use BFS_GRAPH_SORT_ROWS)",
                                     (long long)v);
    }
    if (check_symmetry) {
        for (int64_t v = 0; v < n; ++v)
            for (int64_t j = off[v]; j < off[v + 1]; ++j) {
                const int32_t u = col[j];
                const int32_t *b = col + off[u], *e = col + off[u + 1];
                if (!std::binary_search(b, e, (int32_t)v))
                    return set_error(BFS_E_INVALID, "edge %lld -> %d has no reverse entry",
                                     (long long)v, u);
            }
    }
    return BFS_OK;
}

int validate_options(const bfs_options &o)
{
    if (o.rule < BFS_RULE_EDGES || o.rule > BFS_RULE_BOTTOMUP)
        return set_error(BFS_E_INVALID, "unknown rule %d", o.rule);
    if (o.alpha <= 0 || o.beta <= 0) return set_error(BFS_E_INVALID, "alpha and beta must be > 0");
    if (o.probe_k < 0 || o.probe_k > 64) return set_error(BFS_E_INVALID, "probe_k must be in [0, 64]");
    // the flattened expansion sums 64 degrees in 32 bits
    if (o.td_hub_degree < kHubDegree || o.td_hub_degree > (1 << 24))
        return set_error(BFS_E_INVALID, "td_hub_degree must be in [%d, 2^24]", kHubDegree);
    if (o.grid_blocks < 0) return set_error(BFS_E_INVALID, "grid_blocks < 0");
    if (o.words_per_wave < 0 || o.words_per_wave > 64 || (o.words_per_wave & (o.words_per_wave - 1)))
        return set_error(BFS_E_INVALID, "words_per_wave must be 0 or a power of two <= 64");
    if (o.layers_per_launch < 0 || o.layers_per_launch > 4096)
        return set_error(BFS_E_INVALID, "layers_per_launch must be in [0, 4096]");
    if (o.td_binned < -1 || o.td_binned > 1) return set_error(BFS_E_INVALID, "td_binned must be -1, 0 or 1");
    if (o.first_writer < 0 || o.first_writer > 1) return set_error(BFS_E_INVALID, "first_writer must be 0 or 1");
    if (o.bu_serial_probes < -1 || o.bu_serial_probes > 1)
        return set_error(BFS_E_INVALID, "bu_serial_probes must be -1, 0 or 1");
    if (o.td_queue < -1 || o.td_queue > 2) return set_error(BFS_E_INVALID, "td_queue must be -1, 0, 1 or 2");
    if (o.alpha_binned < 0) return set_error(BFS_E_INVALID, "alpha_binned must be >= 0");
    if (o.bu_filter < -1 || o.bu_filter > 1) return set_error(BFS_E_INVALID, "bu_filter must be -1, 0 or 1");
    if (o.count_work < 0 || o.count_work > 1) return set_error(BFS_E_INVALID, "count_work must be 0 or 1");
    if (o.td_hub_list < -1 || o.td_hub_list > 4)
        return set_error(BFS_E_INVALID, "td_hub_list must be in [-1, 4]");
    if (o.graph_launch < 0 || o.graph_launch > 1 || o.profile_layers < 0 || o.profile_layers > 1 ||
        o.async < 0 || o.async > 1 || o.out_on_device < 0 || o.out_on_device > 1)
        return set_error(BFS_E_INVALID, "flag options must be 0 or 1");
    return BFS_OK;
}

// ------------------------------------------------------------------ workspace
Workspace::~Workspace()
{
    if (dbuf) hipFree(dbuf);
    if (bin_buf) hipFree(bin_buf);
    if (q_buf) hipFree(q_buf);
    if (pstat) hipFree(pstat);
    if (hq_buf) hipFree(hq_buf);
    if (out_tmp) hipFree(out_tmp);
    if (h_ctrl) hipHostFree(h_ctrl);
    if (h_trace) hipHostFree(h_trace);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    for (hipEvent_t e : layer_ev) hipEventDestroy(e);
    for (auto &kv : replays) {
        if (kv.second.exec) hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) hipGraphDestroy(kv.second.graph);
    }
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static size_t workspace_bytes(long long W)
{
    return align256((size_t)W * 8) + align256((size_t)W * 8 * 3) + align256(sizeof(Ctrl)) +
           align256((size_t)kTraceCap * sizeof(LayerRec)) + align256((size_t)3 * kFilterWords * 4);
}

int get_workspace(Graph *g, void *stream, Workspace **out)
{
    std::lock_guard<std::mutex> lk(g->mu);
    auto it = g->ws.find(stream);
    if (it != g->ws.end()) {
        *out = it->second.get();
        return BFS_OK;
    }
    std::unique_ptr<Workspace> w(new (std::nothrow) Workspace());
    if (!w) return set_error(BFS_E_NOMEM, "host allocation");
    hipError_t e;
    if ((e = hipHostMalloc((void **)&w->h_ctrl, sizeof(Ctrl), hipHostMallocDefault)) != hipSuccess)
        return hip_fail(e, "pinned control block");
    if ((e = hipHostMalloc((void **)&w->h_trace, kTraceCap * sizeof(LayerRec), hipHostMallocDefault)) !=
        hipSuccess)
        return hip_fail(e, "pinned trace");
    // timing-only events (read after a stream synchronize): recorded without
    // a system-scope fence, so no cache write-back and invalidate lands in
    // the window they measure
    if ((e = hipEventCreateWithFlags(&w->e0, hipEventDisableSystemFence)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&w->e1, hipEventDisableSystemFence)) != hipSuccess)
        return hip_fail(e, "event");
    const long long W = g->W;
    w->bytes = workspace_bytes(W);
    if ((e = hipMalloc(&w->dbuf, w->bytes)) != hipSuccess) return hip_fail(e, "workspace allocation");
    char *b = (char *)w->dbuf;
    size_t o = 0;
    w->vis = (unsigned long long *)(b + o);  o += align256((size_t)W * 8);
    w->bm = (unsigned long long *)(b + o);   o += align256((size_t)W * 8 * 3);
    w->ctrl = (Ctrl *)(b + o);               o += align256(sizeof(Ctrl));
    w->trace = (LayerRec *)(b + o);          o += align256((size_t)kTraceCap * sizeof(LayerRec));
    w->filt = (unsigned *)(b + o);
    // the workspace is used on `stream` only: a clear ordered on it suffices
    // (no device-wide wait, which would stall the other streams' work)
    if ((e = launch_zero(w->ctrl, align256(sizeof(Ctrl)), (hipStream_t)stream)) != hipSuccess)
        return hip_fail(e, "workspace init");
    *out = w.get();
    g->ws[stream] = std::move(w);
    return BFS_OK;
}

// Reads (and clears) the failure record that the finishers of asynchronous
// traversals keep in a workspace's control block.
template <class W_, class C_>
static int take_async_errors(W_ *w, C_ *h_ctrl, C_ *d_ctrl, hipStream_t s, unsigned *runs, unsigned *bits)
{
    std::lock_guard<std::mutex> wl(w->mu);
    hipError_t e;
    if ((e = hipMemcpyAsync(&h_ctrl->err_runs, &d_ctrl->err_runs, 2 * sizeof(unsigned), hipMemcpyDeviceToHost,
                            s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "reading the failure record");
    if (h_ctrl->err_runs == 0) return BFS_OK;
    *runs += h_ctrl->err_runs;
    *bits |= h_ctrl->err_bits;
    if ((e = hipMemsetAsync(&d_ctrl->err_runs, 0, 2 * sizeof(unsigned), s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "clearing the failure record");
    return BFS_OK;
}

int check_async_errors(Graph *g, void *stream)
{
    Workspace *w = nullptr;
    BatchWorkspace *bw = nullptr;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        auto it = g->ws.find(stream);
        if (it != g->ws.end()) w = it->second.get();
        auto jt = g->bws.find(stream);
        if (jt != g->bws.end()) bw = jt->second.get();
    }
    hipStream_t s = (hipStream_t)stream;
    unsigned runs = 0, bits = 0;
    int rc;
    if (w && (rc = take_async_errors(w, w->h_ctrl, w->ctrl, s, &runs, &bits))) return rc;
    if (bw && (rc = take_async_errors(bw, bw->h_ctrl, bw->ctrl, s, &runs, &bits))) return rc;
    if (runs)
        return set_error(BFS_E_DEVICE,
                         "%u asynchronous traversal(s) on this stream failed a device-side check "
                         "(status bits 0x%x; 0x100: did not end normally)",
                         runs, bits);
    return BFS_OK;
}

size_t Workspace::held() const
{
    return (dbuf ? bytes : 0) + (bin_buf ? bin_bytes : 0) + (q_buf ? q_bytes : 0) + (hq_buf ? hq_bytes : 0) +
           (out_tmp ? (size_t)(out_tmp_n + 64) * 8 : 0) + (pstat ? (size_t)kTraceCap * kCounts * 8 : 0);
}

size_t held_bytes(Graph *g, void *stream, size_t *single, size_t *batch)
{
    std::lock_guard<std::mutex> lk(g->mu);
    size_t a = 0, b = 0;
    auto it = g->ws.find(stream);
    if (it != g->ws.end()) a = it->second->held();
    auto jt = g->bws.find(stream);
    if (jt != g->bws.end()) b = jt->second->held();
    if (single) *single = a;
    if (batch) *batch = b;
    return a + b;
}

void release_workspaces(Graph *g, void *stream)
{
    std::unique_ptr<Workspace> a;
    std::unique_ptr<BatchWorkspace> b;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        auto it = g->ws.find(stream);
        if (it != g->ws.end()) {
            a = std::move(it->second);
            g->ws.erase(it);
        }
        auto jt = g->bws.find(stream);
        if (jt != g->bws.end()) {
            b = std::move(jt->second);
            g->bws.erase(jt);
        }
    }
    // the destructors free the device memory outside the graph's lock
}

// Buckets of the binned top-down step, allocated with the first run that may
// use them: counts, offsets and cursors per tile, and up to min(nnz, 2^28)
// (parent, vertex) pairs.
static size_t bin_bytes(const Graph *g)
{
    const long long cap = std::max<long long>(1, std::min<long long>(g->nnz, 1LL << 28));
    return 3 * align256((size_t)(g->nbins + 1) * 4) + (size_t)cap * 8;
}

static int ensure_bins(Graph *g, Workspace *w, hipStream_t s)
{
    if (w->bin_buf) return BFS_OK;
    const long long cap = std::max<long long>(1, std::min<long long>(g->nnz, 1LL << 28));
    const size_t a = align256((size_t)(g->nbins + 1) * 4);
    const size_t bytes = bin_bytes(g);
    hipError_t e;
    if ((e = hipMalloc(&w->bin_buf, bytes)) != hipSuccess) return hip_fail(e, "binned top-down buckets");
    w->bin_bytes = bytes;
    char *b = (char *)w->bin_buf;
    w->bin_cnt = (int *)b;
    w->bin_off = (int *)(b + a);
    w->bin_cur = (int *)(b + 2 * a);
    w->bin_pairs = (unsigned long long *)(b + 3 * a);
    w->bin_cap = cap;
    if ((e = launch_zero(w->bin_cnt, a, s)) != hipSuccess) return hip_fail(e, "bucket init");
    return BFS_OK;
}

// Library defaults of the queue options (option value 0), from A/B runs on
// MI355X (harmonic-mean GTEPS, 64 roots at SCALE 20 and 22, 16 at SCALE 26):
//  * frontier queues lose everywhere: appends to a queue's one tail
//    serialise (top-down queues: SCALE 20 147 -> 129, SCALE 26 426 -> 418;
//    every layer: 50 and 264), and a top-down layer's bitmap scan is cheap;
//  * hub lists written by every step cost more in the big layers than they
//    save (SCALE 20 101, SCALE 26 427), but the list of layer 0 for layer 1
//    removes layer 1's scan of the hub table: SCALE 26 426 -> 437, SCALE 22
//    296 -> 297, SCALE 20 146 -> 143.  So it is on where the table is large
//    (graphs in the wide build of the layer kernel).
constexpr int kDefaultQueueMode = QM_OFF;
// Membership filters of small frontiers on by default.
constexpr bool kDefaultFilter = true;

void queue_modes(const Graph *g, const bfs_options &opt, int *td_queue, int *hub_list)
{
    *td_queue = opt.td_queue == 0 ? kDefaultQueueMode : opt.td_queue < 0 ? QM_OFF : opt.td_queue;
    *hub_list = opt.td_hub_list == 0 ? (g->wide ? HL_LAYER0 : HL_OFF)
                                     : opt.td_hub_list < 0 ? HL_OFF : opt.td_hub_list;
}

size_t queue_bytes(const Graph *g, bool queues, bool hub_lists)
{
    size_t b = 0;
    if (queues) b += 2 * align256((size_t)g->n * 4);
    if (hub_lists) b += 2 * align256((size_t)std::max<long long>(g->n_hub, 1) * sizeof(Item));
    return b;
}

// Frontier queues and hub lists, allocated with the first run that uses them.
static int ensure_queues(Graph *g, Workspace *w, bool queues, bool hub_lists)
{
    hipError_t e;
    if (queues && !w->q_buf) {
        const size_t a = align256((size_t)g->n * 4);
        if ((e = hipMalloc(&w->q_buf, 2 * a)) != hipSuccess) return hip_fail(e, "frontier queues");
        w->q_bytes = 2 * a;
        w->q[0] = (int *)w->q_buf;
        w->q[1] = (int *)((char *)w->q_buf + a);
    }
    if (hub_lists && !w->hq_buf) {
        const long long cap = std::max<long long>(g->n_hub, 1);
        const size_t a = align256((size_t)cap * sizeof(Item));
        if ((e = hipMalloc(&w->hq_buf, 2 * a)) != hipSuccess) return hip_fail(e, "hub lists");
        w->hq_bytes = 2 * a;
        w->hq[0] = (Item *)w->hq_buf;
        w->hq[1] = (Item *)((char *)w->hq_buf + a);
        w->hq_cap = g->n_hub;
    }
    return BFS_OK;
}

// ------------------------------------------------------------------ launch
void fill_params(const Graph *g, const Workspace *w, const bfs_options &opt, Params *P)
{
    std::memset(P, 0, sizeof *P);
    P->n = g->n;
    P->nnz = g->nnz;
    P->W = g->W;
    P->off = g->d_off;
    P->col = g->d_col;
    P->iso = g->d_iso;
    P->deg = g->d_deg;
    P->slab = g->d_slab;
    P->slab_k = g->slab_k;
    P->chunk_log2 = kChunkLog2;
    P->hub = g->d_hub;
    P->n_hub = g->n_hub;
    P->hub_deg = std::max(g->hub_deg, opt.td_hub_degree);
    P->probe_k = opt.probe_k;
    P->wpg = opt.words_per_wave > 0 ? opt.words_per_wave : g->wpg_default;
    // top-down work is per frontier vertex, so its scan uses wide tasks: a
    // sparse frontier then costs one load per 64 words
    P->wpg_td = 64;
    P->vis = w->vis;
    P->bm = w->bm;
    P->ctrl = w->ctrl;
    P->trace = w->trace;
    P->filt = w->filt;
    // filters are built into the wide layer kernel only (graphs whose frontier
    // bitmap does not fit in the L2)
    P->use_filter = g->wide && (opt.bu_filter > 0 || (opt.bu_filter == 0 && kDefaultFilter));
    P->pstat = w->pstat;
    P->count = opt.count_work && w->pstat ? 1 : 0;
    P->trace_cap = w->trace ? kTraceCap : 0;   // no trace without a buffer for it
    P->rule = opt.rule;
    P->alpha = opt.alpha;
    P->beta = opt.beta;
    P->alpha_bin = opt.alpha_binned > 0 ? opt.alpha_binned : opt.alpha;
    P->first_writer = opt.first_writer;
    P->async_run = opt.async;
    P->serial_probes = opt.bu_serial_probes > 0 || (opt.bu_serial_probes == 0 && g->n >= (1LL << 24));
    P->wide = g->wide ? 1 : 0;
    P->nbins = g->nbins;
    P->bin_log2 = kBinLog2;
    P->bin_cnt = w->bin_cnt;
    P->bin_off = w->bin_off;
    P->bin_cur = w->bin_cur;
    P->bin_pairs = w->bin_pairs;
    P->bin_cap = w->bin_pairs ? w->bin_cap : 0;
    P->bin_min_edges = opt.td_binned > 0 ? 1 : (1LL << 22);
    int qm = QM_OFF, hl = 0;
    queue_modes(g, opt, &qm, &hl);
    // without its buffers a mode stays off (the no-allocation entry point)
    if (!w->q[0]) qm = QM_OFF;
    if (!w->hq[0]) hl = 0;
    P->td_queue = qm;
    P->q0 = w->q[0];
    P->q1 = w->q[1];
    P->q_cap = w->q[0] ? g->n : 0;
    P->hub_list = hl;
    P->hq0 = w->hq[0];
    P->hq1 = w->hq[1];
    P->hq_cap = w->hq_cap;
    P->q_write = 0;
    P->h_write = 0;
}

size_t single_run_bytes(Graph *g, void *stream, const bfs_options &opt)
{
    std::lock_guard<std::mutex> lk(g->mu);
    auto it = g->ws.find(stream);
    const Workspace *w = it != g->ws.end() ? it->second.get() : nullptr;
    const bool bins = g->nbins <= kMaxBins && (opt.td_binned > 0 || (opt.td_binned == 0 && g->bin_auto));
    int qm = QM_OFF, hl = 0;
    queue_modes(g, opt, &qm, &hl);
    // each part: what the workspace holds, or what the run allocates for it
    size_t b = w && w->dbuf ? w->bytes : workspace_bytes(g->W);
    b += w && w->bin_buf ? w->bin_bytes : (bins ? bin_bytes(g) : 0);
    b += w && w->q_buf ? w->q_bytes : queue_bytes(g, qm != QM_OFF, false);
    b += w && w->hq_buf ? w->hq_bytes : queue_bytes(g, false, hl != 0);
    const size_t tmp = w && w->out_tmp ? (size_t)(w->out_tmp_n + 64) * 8 : 0;
    b += opt.out_on_device ? tmp : std::max(tmp, (size_t)(g->n + 64) * 8);
    b += (w && w->pstat) || opt.count_work ? (size_t)kTraceCap * kCounts * 8 : 0;
    return b;
}

int enqueue_traversal(Graph *g, Workspace *w, const bfs_options &opt, int root, int *lvl, int *par,
                      hipStream_t s, int *layers_enqueued, bool profile, int *layer0_kernel)
{
    // binned top-down: allowed on the layers after which its kernels are enqueued
    const bool bins = g->nbins <= kMaxBins && (opt.td_binned > 0 || (opt.td_binned == 0 && g->bin_auto));
    if (bins) {
        const int rc = ensure_bins(g, w, s);
        if (rc) return rc;
    }
    if (!w->no_alloc) {
        int qm = QM_OFF, hl = 0;
        queue_modes(g, opt, &qm, &hl);
        const int rc = ensure_queues(g, w, qm != QM_OFF, hl != 0);
        if (rc) return rc;
    }
    Params P;
    fill_params(g, w, opt, &P);
    P.root = root;
    P.level = lvl;
    P.parent = par;
    P.fail_injected = root == g->fail_root;
    const int grid = opt.grid_blocks > 0 ? opt.grid_blocks : g->grid_default;
    const int L = opt.layers_per_launch > 0 ? opt.layers_per_launch : g->depth.typical.load();
    hipError_t e;
    if (profile) {
        while ((int)w->layer_ev.size() < 2 * L) {
            hipEvent_t ev;
            if ((e = hipEventCreateWithFlags(&ev, hipEventDisableSystemFence)) != hipSuccess)
                return hip_fail(e, "event");
            w->layer_ev.push_back(ev);
        }
    }
    // layer 0 is the root's own row: for a root of small degree it runs in the
    // initialisation kernel (each block takes the neighbours in its own range)
    // or, where that cannot be used, in one block instead of the grid
    const bool small_root = g->h_deg[root] <= kRootKernelDegree;
    const long long per = (g->W + grid - 1) / grid;
    const bool fused = small_root && per <= kFuseWords && w->counters_zero;
    w->counters_zero = false;
    if ((e = fused ? launch_init_root(P, grid, (int)per, s) : launch_init(P, grid, s)) != hipSuccess)
        return hip_fail(e, "init launch");
    for (int i = 0; i < L; ++i) {
        if (profile && (e = hipEventRecord(w->layer_ev[2 * i], s)) != hipSuccess) return hip_fail(e, "event");
        if (i == 0 && small_root) {
            if (!fused && (e = launch_root(P, s)) != hipSuccess) return hip_fail(e, "root launch");
            if (profile && (e = hipEventRecord(w->layer_ev[1], s)) != hipSuccess) return hip_fail(e, "event");
            continue;
        }
        const int allow = bins && (opt.td_binned > 0 || (i >= 1 && i <= 5));
        if ((e = launch_layer(P, i, allow, grid, s)) != hipSuccess) return hip_fail(e, "layer launch");
        if (allow) {
            if ((e = launch_bin_scan(P, i, s)) != hipSuccess ||
                (e = launch_bin_scatter(P, i, grid, s)) != hipSuccess ||
                (e = launch_bin_reduce(P, i, 2 * g->cus, s)) != hipSuccess)
                return hip_fail(e, "binned top-down launch");
        }
        if (profile && (e = hipEventRecord(w->layer_ev[2 * i + 1], s)) != hipSuccess) return hip_fail(e, "event");
    }
    if ((e = launch_finish(P, s)) != hipSuccess) return hip_fail(e, "finisher launch");
    w->counters_zero = true;
    // launches of the layer kernel itself
    if (layers_enqueued) *layers_enqueued = small_root ? L - 1 : L;
    if (layer0_kernel) *layer0_kernel = fused ? 2 : small_root ? 1 : 0;
    return BFS_OK;
}

// hipGraph replay of the launch sequence of enqueue_traversal: the
// initialisation kernel (fused with layer 0 for a root of small degree, as
// in a direct launch), the layer kernels with the binned top-down kernels
// after the layers that may bin, and the finisher.  One graph is built per
// workspace, option set and form of layer 0 (the host knows the root's
// degree); a run rewrites only the initialisation node's arguments (root and
// output pointers), which the other kernels pick up from the control block.
int enqueue_traversal_graph(Graph *g, Workspace *w, const bfs_options &opt, int root, int *lvl,
                            int *par, hipStream_t s, int *layers_enqueued, int *layer0_kernel)
{
    const bool bins = g->nbins <= kMaxBins && (opt.td_binned > 0 || (opt.td_binned == 0 && g->bin_auto));
    if (bins) {
        const int rc = ensure_bins(g, w, s);
        if (rc) return rc;
    }
    {
        int qm = QM_OFF, hl = 0;
        queue_modes(g, opt, &qm, &hl);
        const int rc = ensure_queues(g, w, qm != QM_OFF, hl != 0);
        if (rc) return rc;
    }
    Params P;
    fill_params(g, w, opt, &P);
    const int grid = opt.grid_blocks > 0 ? opt.grid_blocks : g->grid_default;
    const int L = opt.layers_per_launch > 0 ? opt.layers_per_launch : g->depth.typical.load();
    const long long per = (g->W + grid - 1) / grid;
    // layer 0 inside the initialisation kernel needs every counter slot at
    // zero, which a replayed finisher leaves behind
    const bool fused = g->h_deg[root] <= kRootKernelDegree && per <= kFuseWords && w->counters_zero;
    char key[200];
    snprintf(key, sizeof key, "%d/%d/%d/%d/%d/%d/%d/%d/%d/%d/%d/%d/%d/%lld/%d/%d/%d/%d", opt.rule, opt.alpha,
             opt.beta, opt.probe_k, P.wpg, P.wpg_td, P.hub_deg, P.first_writer, P.serial_probes, grid, L,
             P.td_queue, P.hub_list, P.alpha_bin, P.use_filter, opt.td_binned, fused ? 1 : 0, bins ? 1 : 0);
    hipError_t e;
    int per_arg = (int)per;
    auto it = w->replays.find(key);
    if (it == w->replays.end()) {
        Workspace::Replay R;
        R.params = P;
        R.params.root = root;
        R.params.level = lvl;
        R.params.parent = par;
        R.fused = fused;
        if ((e = hipGraphCreate(&R.graph, 0)) != hipSuccess) return hip_fail(e, "graph create");
        // a graph that could not be built completely is destroyed
        auto fail = [&](hipError_t err, const char *what) {
            hipGraphDestroy(R.graph);
            return hip_fail(err, what);
        };
        std::vector<int> layer_idx(L);
        for (int i = 0; i < L; ++i) layer_idx[i] = i;
        hipGraphNode_t prev = nullptr;
        hipKernelNodeParams kp;
        std::memset(&kp, 0, sizeof kp);
        void *init_args[] = {&R.params};
        void *init_fused_args[] = {&R.params, &per_arg};
        kp.func = fused ? kernel_ptr_init_root() : kernel_ptr_init();
        kp.gridDim = dim3(grid);
        kp.blockDim = dim3(kBlock);
        kp.kernelParams = fused ? init_fused_args : init_args;
        if ((e = hipGraphAddKernelNode(&R.init, R.graph, nullptr, 0, &kp)) != hipSuccess)
            return fail(e, "graph init node");
        prev = R.init;
        auto add = [&](void *fn, dim3 gd, dim3 bd, void **args) -> hipError_t {
            hipKernelNodeParams np;
            std::memset(&np, 0, sizeof np);
            np.func = fn;
            np.gridDim = gd;
            np.blockDim = bd;
            np.kernelParams = args;
            hipGraphNode_t node;
            const hipError_t r = hipGraphAddKernelNode(&node, R.graph, &prev, 1, &np);
            if (r == hipSuccess) prev = node;
            return r;
        };
        std::vector<int> allow(L);
        for (int i = fused ? 1 : 0; i < L; ++i) {
            allow[i] = bins && (opt.td_binned > 0 || (i >= 1 && i <= 5));
            void *args[] = {&R.params, &layer_idx[i], &allow[i]};
            if ((e = add(kernel_ptr_layer(R.params.wide != 0, layer_build(R.params, i), layer_filter(R.params, i)),
                         dim3(grid), dim3(kBlock), args)) != hipSuccess)
                return fail(e, "graph layer node");
            if (allow[i]) {
                void *bargs[] = {&R.params, &layer_idx[i]};
                if ((e = add(kernel_ptr_bin_scan(), dim3(1), dim3(kFinishBlock), bargs)) != hipSuccess ||
                    (e = add(kernel_ptr_bin_scatter(), dim3(grid), dim3(kBlock), bargs)) != hipSuccess ||
                    (e = add(kernel_ptr_bin_reduce(), dim3(2 * g->cus), dim3(kReduceBlockThreads), bargs)) !=
                        hipSuccess)
                    return fail(e, "graph binned nodes");
            }
        }
        void *fin_args[] = {&R.params};
        if ((e = add(kernel_ptr_finish(finish_build(R.params)), dim3(1), dim3(kFinisherBlock), fin_args)) !=
            hipSuccess)
            return fail(e, "graph finisher node");
        if ((e = hipGraphInstantiate(&R.exec, R.graph, nullptr, nullptr, 0)) != hipSuccess)
            return fail(e, "graph instantiate");
        it = w->replays.emplace(key, R).first;
    }
    Workspace::Replay &R = it->second;
    R.params.root = root;
    R.params.level = lvl;
    R.params.parent = par;
    R.params.async_run = opt.async;
    R.params.fail_injected = root == g->fail_root;
    void *init_args[] = {&R.params};
    void *init_fused_args[] = {&R.params, &per_arg};
    hipKernelNodeParams kp;
    std::memset(&kp, 0, sizeof kp);
    kp.func = R.fused ? kernel_ptr_init_root() : kernel_ptr_init();
    kp.gridDim = dim3(grid);
    kp.blockDim = dim3(kBlock);
    kp.kernelParams = R.fused ? init_fused_args : init_args;
    if ((e = hipGraphExecKernelNodeSetParams(R.exec, R.init, &kp)) != hipSuccess)
        return hip_fail(e, "graph update");
    w->counters_zero = false;
    if ((e = hipGraphLaunch(R.exec, s)) != hipSuccess) return hip_fail(e, "graph launch");
    w->counters_zero = true;   // the replayed finisher clears them
    if (layers_enqueued) *layers_enqueued = R.fused ? L - 1 : L;
    if (layer0_kernel) *layer0_kernel = R.fused ? 2 : 0;
    return BFS_OK;
}


// Adaptive layer count: the deepest of the last 16 traversals.  A traversal of
// that depth ends in the single-block finisher, which only has to see the
// empty frontier; deeper ones are finished there.
void DepthTracker::note(int nlayers)
{
    const unsigned p = pos.fetch_add(1) % 16;
    recent[p].store(nlayers);
    int mx = 0;
    for (int i = 0; i < 16; ++i) mx = std::max(mx, recent[i].load());
    typical.store(std::min(std::max(mx, 2), 64));
}

}  // namespace hybfs

using namespace hybfs;

// ====================================================================== ABI
extern "C" {

const char *bfs_last_error(void) { return last_error(); }

void bfs_options_init(bfs_options *opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof *opt);
    opt->rule = BFS_RULE_EDGES;
    opt->alpha = 14;
    opt->beta = 24;
    opt->probe_k = 8;
    opt->td_hub_degree = kHubDegree;
    opt->td_binned = 0;
}

int bfs_graph_create(int64_t n, int64_t nnz, const int64_t *row_offsets, const int32_t *col_indices,
                     uint32_t flags, bfs_graph_t *out)
{
    clear_error();
    if (!out) return set_error(BFS_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > 0x7FFFFFFFLL) return set_error(BFS_E_INVALID, "n = %lld out of [1, 2^31-1]", (long long)n);
    if (nnz < 0) return set_error(BFS_E_INVALID, "nnz < 0");
    if (!row_offsets || (nnz > 0 && !col_indices)) return set_error(BFS_E_INVALID, "NULL CSR array");
    if (flags & ~(uint32_t)(BFS_GRAPH_DEVICE_INPUT | BFS_GRAPH_ASSUME_VALID | BFS_GRAPH_CHECK_SYMMETRY |
                            BFS_GRAPH_SORT_ROWS))
        return set_error(BFS_E_INVALID, "unknown flag bits 0x%x", flags);

    const bool dev_in = flags & BFS_GRAPH_DEVICE_INPUT;
    const bool sort_rows = flags & BFS_GRAPH_SORT_ROWS;
    const bool validate = !(flags & BFS_GRAPH_ASSUME_VALID);
    const bool symmetry = flags & BFS_GRAPH_CHECK_SYMMETRY;

    // Host views of the CSR (copies only where needed).
    std::vector<int64_t> h_off_store;
    std::vector<int32_t> h_col_store;
    const int64_t *h_off = row_offsets;
    const int32_t *h_col = col_indices;
    if (dev_in) {
        try {
            h_off_store.resize((size_t)n + 1);
            if (validate || sort_rows || symmetry) h_col_store.resize((size_t)nnz);
        } catch (...) {
            return set_error(BFS_E_NOMEM, "host staging");
        }
        hipError_t e = hipMemcpy(h_off_store.data(), row_offsets, (n + 1) * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "reading device row_offsets");
        if (!h_col_store.empty()) {
            e = hipMemcpy(h_col_store.data(), col_indices, nnz * 4, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_fail(e, "reading device col_indices");
        }
        h_off = h_off_store.data();
        h_col = h_col_store.empty() ? nullptr : h_col_store.data();
    }
    if (h_off[0] != 0 || h_off[n] != nnz)
        return set_error(BFS_E_INVALID, "row_offsets must start at 0 and end at nnz");
    for (int64_t v = 0; v < n; ++v)
        if (h_off[v + 1] < h_off[v])
            return set_error(BFS_E_INVALID, "row_offsets decreases at vertex %lld", (long long)v);
    if (sort_rows) {
        if (h_col_store.empty() && nnz > 0) {
            try {
                h_col_store.assign(col_indices, col_indices + nnz);
            } catch (...) {
                return set_error(BFS_E_NOMEM, "host copy for sorting");
            }
        }
        for (int64_t v = 0; v < n; ++v)
            std::sort(h_col_store.begin() + h_off[v], h_col_store.begin() + h_off[v + 1]);
        h_col = h_col_store.empty() ? nullptr : h_col_store.data();
    }
    // a symmetry check needs in-range, sorted rows: it implies the full check
    if (validate || symmetry) {
        int rc = check_csr(n, nnz, h_off, h_col, true, symmetry);
        if (rc) return rc;
    }

    std::unique_ptr<Graph> g(new (std::nothrow) Graph());
    if (!g) return set_error(BFS_E_NOMEM, "host allocation");
    hipError_t e = hipGetDevice(&g->dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    g->n = n;
    g->nnz = nnz;
    g->W = (n + 63) >> 6;
    // per-vertex data every traversal reads: degrees and the position-major
    // slab of each row's first slab_k entries (-1 past the end of the row)
    g->slab_k = n <= (1LL << 25) ? 4 : 2;
    std::vector<int32_t> deg, slab;
    try {
        deg.resize((size_t)n);
        slab.assign((size_t)n * g->slab_k, -1);
    } catch (...) {
        return set_error(BFS_E_NOMEM, "host staging of per-vertex data");
    }
    int64_t iso = 0, maxd = 0;
    for (int64_t v = 0; v < n; ++v) {
        const int64_t dv = h_off[v + 1] - h_off[v];
        if (dv > 0x7FFFFFFF) return set_error(BFS_E_INVALID, "degree of vertex %lld exceeds 2^31-1", (long long)v);
        deg[v] = (int32_t)dv;
        iso += dv == 0;
        maxd = std::max(maxd, dv);
    }
    if (nnz > 0) {
        // the columns may only be on the device (unvalidated device input)
        std::vector<int32_t> tmp;
        const int32_t *cols = h_col;
        if (!cols) {
            try {
                tmp.resize((size_t)nnz);
            } catch (...) {
                return set_error(BFS_E_NOMEM, "host staging of columns");
            }
            if ((e = hipMemcpy(tmp.data(), col_indices, nnz * 4, hipMemcpyDeviceToHost)) != hipSuccess)
                return hip_fail(e, "reading device col_indices");
            cols = tmp.data();
        }
        for (int64_t v = 0; v < n; ++v)
            for (int p = 0; p < g->slab_k && p < deg[v]; ++p) slab[(size_t)p * n + v] = cols[h_off[v] + p];
    }
    g->isolated = iso;
    g->max_degree = maxd;
    // top-down hub table: every 256-edge chunk of each vertex above hub_deg
    std::vector<Item> hub;
    {
        const int64_t H = kHubDegree;
        g->hub_deg = (int)H;
        for (int64_t v = 0; v < n; ++v)
            if (deg[v] > H) {
                const int64_t k = ((int64_t)deg[v] + (1 << kChunkLog2) - 1) >> kChunkLog2;
                for (int64_t c = 0; c < k; ++c) hub.push_back(Item{(int)v, (int)c});
            }
        g->n_hub = (long long)hub.size();
    }
    // the same rows in segments of 2^kSegLog2 chunks (batched bottom-up
    // scans), numbered row-major, listed by segment number so that a row's
    // earlier segments are scanned (and publish their finds) first
    std::vector<HSeg> hseg;
    {
        long long id = 0, first = 0;
        for (size_t i = 0; i < hub.size(); ++i) {
            if (hub[i].chunk == 0) first = id;
            if ((hub[i].chunk & ((1 << kSegLog2) - 1)) == 0) {
                hseg.push_back(HSeg{hub[i].u, hub[i].chunk >> kSegLog2, first});
                ++id;
            }
        }
        std::stable_sort(hseg.begin(), hseg.end(), [](const HSeg &a, const HSeg &b) { return a.seg < b.seg; });
    }
    g->n_hseg = (long long)hseg.size();

    if ((e = hipMalloc(&g->d_off, (n + 1) * 8)) != hipSuccess) return hip_fail(e, "graph offsets");
    if ((e = hipMalloc(&g->d_col, std::max<int64_t>(nnz, 1) * 4)) != hipSuccess) return hip_fail(e, "graph columns");
    if ((e = hipMalloc(&g->d_iso, g->W * 8)) != hipSuccess) return hip_fail(e, "graph bitmap");
    if ((e = hipMalloc(&g->d_deg, n * 4)) != hipSuccess) return hip_fail(e, "degrees");
    if ((e = hipMalloc(&g->d_slab, n * 4 * g->slab_k)) != hipSuccess) return hip_fail(e, "slab");
    if ((e = hipMalloc(&g->d_hub, std::max<size_t>(hub.size(), 1) * sizeof(Item))) != hipSuccess)
        return hip_fail(e, "hub table");
    if (!hub.empty() &&
        (e = hipMemcpy(g->d_hub, hub.data(), hub.size() * sizeof(Item), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "upload hub table");
    if ((e = hipMalloc(&g->d_hseg, std::max<size_t>(hseg.size(), 1) * sizeof(HSeg))) != hipSuccess)
        return hip_fail(e, "hub segment table");
    if (!hseg.empty() &&
        (e = hipMemcpy(g->d_hseg, hseg.data(), hseg.size() * sizeof(HSeg), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "upload hub segment table");
    e = hipMemcpy(g->d_off, h_off, (n + 1) * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "upload offsets");
    if (nnz > 0) {
        const bool from_dev = dev_in && h_col == nullptr;
        e = hipMemcpy(g->d_col, from_dev ? col_indices : h_col, nnz * 4,
                      from_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "upload columns");
    }
    if ((e = hipMemcpy(g->d_deg, deg.data(), n * 4, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "upload degrees");
    g->h_deg = std::move(deg);
    if ((e = hipMemcpy(g->d_slab, slab.data(), n * 4 * g->slab_k, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "upload slab");
    if ((e = launch_iso_template(g->d_off, n, g->W, g->d_iso, 0)) != hipSuccess) return hip_fail(e, "iso kernel");
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "graph setup");

    int cus = 0;
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->dev);
    g->wide = n >= kWideMinVertices;
    const int per_cu = layer_blocks_per_cu(g->wide);
    if (per_cu < 1 || cus < 1) return set_error(BFS_E_DEVICE, "occupancy query failed");
    g->cus = cus;
    g->blocks_per_cu = per_cu;
    g->grid_default = std::min(per_cu, g->wide ? kWideBlocksPerCu : kLayerBlocksPerCu) * cus;
    // size a wavefront task so that about two tasks fall on each resident wave
    const long long resident_waves = (long long)g->grid_default * kWavesPerBlock;
    int wpg = 1;
    while (wpg < 64 && (g->W + wpg - 1) / wpg > 2 * resident_waves) wpg <<= 1;
    g->wpg_default = wpg;
    for (int i = 0; i < 16; ++i) {
        g->depth.recent[i].store(9);
        g->batch_depth.recent[i].store(9);
    }
    const int bper_cu = batch_blocks_per_cu();
    if (bper_cu < 1) return set_error(BFS_E_DEVICE, "occupancy query failed");
    g->batch_grid = std::min(bper_cu, 4) * cus;
    g->nbins = (int)((n + (1LL << kBinLog2) - 1) >> kBinLog2);
    g->bin_auto = n >= (1LL << 23) && g->nbins <= kMaxBins;
    if (const char *fr = getenv("HYBFS_TEST_FAIL_ROOT")) g->fail_root = atoi(fr);
    const int pper_cu = batch_pull_blocks_per_cu();
    if (pper_cu < 1) return set_error(BFS_E_DEVICE, "occupancy query failed");
    g->batch_pull_grid = pper_cu * cus;
    *out = reinterpret_cast<bfs_graph_t>(g.release());
    return BFS_OK;
}

int bfs_graph_destroy(bfs_graph_t gh)
{
    clear_error();
    if (!gh) return set_error(BFS_E_INVALID, "NULL graph");
    Graph *g = reinterpret_cast<Graph *>(gh);
    hipDeviceSynchronize();
    for (auto &kv : g->ws) kv.second.reset();
    g->ws.clear();
    for (auto &kv : g->bws) kv.second.reset();
    g->bws.clear();
    if (g->d_off) hipFree(g->d_off);
    if (g->d_col) hipFree(g->d_col);
    if (g->d_iso) hipFree(g->d_iso);
    if (g->d_deg) hipFree(g->d_deg);
    if (g->d_slab) hipFree(g->d_slab);
    if (g->d_hub) hipFree(g->d_hub);
    if (g->d_hseg) hipFree(g->d_hseg);
    delete g;
    return BFS_OK;
}

int bfs_graph_info_get(bfs_graph_t gh, bfs_graph_info *info)
{
    clear_error();
    if (!gh || !info) return set_error(BFS_E_INVALID, "NULL argument");
    Graph *g = reinterpret_cast<Graph *>(gh);
    std::memset(info, 0, sizeof *info);
    info->n = g->n;
    info->nnz = g->nnz;
    info->isolated = g->isolated;
    info->max_degree = g->max_degree;
    info->device_bytes = (g->n + 1) * 8 + g->nnz * 4 + g->W * 8 + g->n * 4 * (1 + g->slab_k) +
                         g->n_hub * (int64_t)sizeof(Item) + g->n_hseg * (int64_t)sizeof(HSeg);
    info->workspace_bytes = (int64_t)workspace_bytes(g->W);
    info->grid_blocks = g->grid_default;
    info->block_threads = kBlock;
    info->slab_k = g->slab_k;
    info->chunk_edges = 1 << kChunkLog2;
    info->hub_degree = g->hub_deg;
    info->hub_chunks = g->n_hub;
    info->typical_layers = g->depth.typical.load();
    info->batch_workspace_bytes = (int64_t)batch_workspace_bytes(g);
    info->layer_kernel_wide = g->wide ? 1 : 0;
    info->reserved = 0;
    return BFS_OK;
}

int bfs_run(bfs_graph_t gh, int32_t root, int32_t *level_out, int32_t *parent_out,
            const bfs_options *opt_in, bfs_stats *stats)
{
    clear_error();
    if (!gh) return set_error(BFS_E_INVALID, "NULL graph");
    Graph *g = reinterpret_cast<Graph *>(gh);
    bfs_options opt;
    if (opt_in) opt = *opt_in;
    else bfs_options_init(&opt);
    int rc = validate_options(opt);
    if (rc) return rc;
    if (root < 0 || (int64_t)root >= g->n)
        return set_error(BFS_E_INVALID, "root %d out of [0, %lld)", root, (long long)g->n);
    if (!level_out || !parent_out) return set_error(BFS_E_INVALID, "NULL output");
    if (opt.async && (!opt.out_on_device || stats))
        return set_error(BFS_E_INVALID, "async runs need device outputs and no stats");
    if (opt.count_work && !stats) return set_error(BFS_E_INVALID, "count_work needs stats");

    Workspace *w = nullptr;
    rc = get_workspace(g, opt.stream, &w);
    if (rc) return rc;
    std::lock_guard<std::mutex> wl(w->mu);
    hipStream_t s = (hipStream_t)opt.stream;
    hipError_t e;
    if (opt.count_work && !w->pstat &&
        (e = hipMalloc(&w->pstat, (size_t)kTraceCap * kCounts * 8)) != hipSuccess)
        return hip_fail(e, "work counters");

    int *lvl = level_out, *par = parent_out;
    if (!opt.out_on_device) {
        if (!w->out_tmp || w->out_tmp_n < g->n) {
            if (w->out_tmp) {
                hipStreamSynchronize(s);
                hipFree(w->out_tmp);
                w->out_tmp = nullptr;
            }
            if ((e = hipMalloc(&w->out_tmp, (g->n + 64) * 8)) != hipSuccess)
                return hip_fail(e, "output staging");
            w->out_tmp_n = g->n;
        }
        lvl = w->out_tmp;
        par = w->out_tmp + ((g->n + 63) & ~63LL);
    }

    const bool profile = opt.profile_layers && stats && !opt.async;
    int launched = 0, layer0 = 0;
    // the traversal's own events only serve stats->device_us: every event
    // record is a marker packet with its own cost on the device
    if (stats && (e = hipEventRecord(w->e0, s)) != hipSuccess) return hip_fail(e, "event record");
    if (!opt.graph_launch || profile)
        rc = enqueue_traversal(g, w, opt, root, lvl, par, s, &launched, profile, &layer0);
    else
        rc = enqueue_traversal_graph(g, w, opt, root, lvl, par, s, &launched, &layer0);
    if (rc) return rc;
    if (stats && (e = hipEventRecord(w->e1, s)) != hipSuccess) return hip_fail(e, "event record");
    if (opt.async) return BFS_OK;

    if ((e = hipMemcpyAsync(w->h_ctrl, w->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "control copy");
    if (!opt.out_on_device) {
        if ((e = hipMemcpyAsync(level_out, lvl, g->n * 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipMemcpyAsync(parent_out, par, g->n * 4, hipMemcpyDeviceToHost, s)) != hipSuccess)
            return hip_fail(e, "copy outputs to host");
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "traversal");
    const Ctrl &c = *w->h_ctrl;
    if (c.done != 1 || c.status != 0) {
        return set_error(BFS_E_DEVICE, "traversal failed a device-side check (done %d, status %d)",
                         c.done, c.status);
    }
    g->depth.note(c.nlayers);
    if (stats) {
        stats->num_layers = c.nlayers;
        stats->reached = c.reached;
        stats->reached_degree_sum = c.reached_deg;
        float ms = 0.f;
        hipEventElapsedTime(&ms, w->e0, w->e1);
        stats->device_us = ms * 1000.0;
        stats->layer_launches = launched;
        stats->layer0_kernel = layer0;
        stats->layer_kernel_us = 0.0;
        // per enqueued layer: layer 0 first (its pair of events brackets the
        // one-block kernel, or nothing when it ran in the initialisation
        // kernel), then one layer-kernel launch each
        const int nev = launched + (layer0 ? 1 : 0);
        std::vector<double> kus(nev, 0.0);
        if (profile) {
            for (int i = 0; i < nev; ++i) {
                float lm = 0.f;
                hipEventElapsedTime(&lm, w->layer_ev[2 * i], w->layer_ev[2 * i + 1]);
                kus[i] = lm * 1000.0;
                if (i > 0 || !layer0) stats->layer_kernel_us += kus[i];
            }
        }
        const int nrec = std::min(c.nlayers, kTraceCap);
        if (stats->layers && stats->capacity > 0 && nrec > 0) {
            const int ncopy = std::min(nrec, stats->capacity);
            e = hipMemcpy(w->h_trace, w->trace, nrec * sizeof(LayerRec), hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_fail(e, "trace copy");
            std::vector<unsigned long long> work;
            if (opt.count_work) {
                work.resize((size_t)ncopy * kCounts);
                e = hipMemcpy(work.data(), w->pstat, work.size() * 8, hipMemcpyDeviceToHost);
                if (e != hipSuccess) return hip_fail(e, "work counter copy");
            }
            for (int i = 0; i < ncopy; ++i) {
                const LayerRec &r = w->h_trace[i];
                bfs_layer_stat &o = stats->layers[i];
                for (int k = 0; k < 6; ++k) o.work[k] = (k < kCounts && !work.empty()) ? (int64_t)work[i * kCounts + k] : 0;
                o.direction = r.dir;
                o.reserved = 0;
                o.n_f = r.n_f;
                o.m_f = r.m_f;
                o.m_u = r.m_u;
                o.v_u = r.v_u;
                o.kernel_us = (profile && i < nev) ? kus[i] : 0.0;
                o.t_us = o.kernel_us;
            }
        }
    }
    return BFS_OK;
}

int bfs_graph_sync(bfs_graph_t gh, void *stream)
{
    clear_error();
    if (!gh) return set_error(BFS_E_INVALID, "NULL graph");
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "stream synchronize");
    return check_async_errors(reinterpret_cast<Graph *>(gh), stream);
}

}  // extern "C"
