// Host side of the batched multi-source traversal (bfs_run_batch).
#include <algorithm>
#include <cstdio>
#include <cstring>

#include "hybfs_internal.h"

namespace hybfs {

BatchWorkspace::~BatchWorkspace()
{
    if (dbuf) hipFree(dbuf);
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

size_t batch_workspace_bytes(const Graph *g)
{
    const long long n = g->n, W = g->W;
    return align256((size_t)n * 8) + align256((size_t)n * 8 * (kBatchHist + 3)) + align256((size_t)W * 8 * 3) +
           align256((size_t)std::max<long long>(g->n_hseg, 1) * 8) + align256(sizeof(BCtrl)) +
           align256((size_t)kTraceCap * sizeof(LayerRec)) + align256(2 * kLanes * sizeof(int *));
}

int get_batch_workspace(Graph *g, void *stream, BatchWorkspace **out)
{
    std::lock_guard<std::mutex> lk(g->mu);
    auto it = g->bws.find(stream);
    if (it != g->bws.end()) {
        *out = it->second.get();
        return BFS_OK;
    }
    std::unique_ptr<BatchWorkspace> w(new (std::nothrow) BatchWorkspace());
    if (!w) return set_error(BFS_E_NOMEM, "host allocation");
    hipError_t e;
    if ((e = hipHostMalloc((void **)&w->h_ctrl, sizeof(BCtrl), hipHostMallocDefault)) != hipSuccess)
        return hip_fail(e, "pinned control block");
    if ((e = hipHostMalloc((void **)&w->h_trace, kTraceCap * sizeof(LayerRec), hipHostMallocDefault)) !=
        hipSuccess)
        return hip_fail(e, "pinned trace");
    if ((e = hipEventCreateWithFlags(&w->e0, hipEventDisableSystemFence)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&w->e1, hipEventDisableSystemFence)) != hipSuccess)
        return hip_fail(e, "event");
    const long long n = g->n, W = g->W;
    w->bytes = batch_workspace_bytes(g);
    if ((e = hipMalloc(&w->dbuf, w->bytes)) != hipSuccess) return hip_fail(e, "batch workspace allocation");
    char *b = (char *)w->dbuf;
    size_t o = 0;
    w->vis = (unsigned long long *)(b + o);  o += align256((size_t)n * 8);
    w->fm = (unsigned long long *)(b + o);   o += align256((size_t)n * 8 * (kBatchHist + 3));
    w->ubm = (unsigned long long *)(b + o);  o += align256((size_t)W * 8 * 3);
    w->sfound = (unsigned long long *)(b + o);  o += align256((size_t)std::max<long long>(g->n_hseg, 1) * 8);
    w->ctrl = (BCtrl *)(b + o);              o += align256(sizeof(BCtrl));
    w->trace = (LayerRec *)(b + o);          o += align256((size_t)kTraceCap * sizeof(LayerRec));
    w->tab = (int **)(b + o);
    // used on `stream` only: a clear ordered on it suffices.  The kept mask
    // slots start clear here; afterwards each level pass clears what it read.
    if ((e = launch_zero(w->ctrl, align256(sizeof(BCtrl)), (hipStream_t)stream)) != hipSuccess ||
        (e = launch_zero(w->fm, align256((size_t)n * 8 * kBatchHist), (hipStream_t)stream)) != hipSuccess)
        return hip_fail(e, "workspace init");
    *out = w.get();
    g->bws[stream] = std::move(w);
    return BFS_OK;
}

static void fill_batch_params(const Graph *g, const BatchWorkspace *w, const bfs_options &opt, int k,
                              BParams *P)
{
    std::memset(P, 0, sizeof *P);
    P->n = g->n;
    P->nnz = g->nnz;
    P->W = g->W;
    P->off = g->d_off;
    P->col = g->d_col;
    P->deg = g->d_deg;
    P->iso = g->d_iso;
    P->hub = g->d_hub;
    P->n_hub = g->n_hub;
    P->hub_log2 = kChunkLog2;
    P->hub_deg = g->hub_deg;
    P->hseg = g->d_hseg;
    P->n_hseg = g->n_hseg;
    P->sfound = w->sfound;
    P->seg_log2 = kSegLog2;
    P->k = k;
    P->rule = opt.rule;
    P->active = k >= 64 ? ~0ull : ((1ull << k) - 1ull);
    P->vis = w->vis;
    P->fm = w->fm;
    P->ubm = w->ubm;
    P->lvl = w->tab;
    P->par = w->tab + kLanes;
    P->ctrl = w->ctrl;
    P->trace = w->trace;
    P->trace_cap = kTraceCap;
    P->wpg = opt.words_per_wave > 0 ? opt.words_per_wave : g->wpg_default;
    P->wpg_td = 64;
    P->alpha = opt.alpha;
    P->beta = opt.beta;
    P->async_run = opt.async;
    P->hist = kBatchHist;
}

static void fill_roots(const Graph *g, const int32_t *roots, int k, RootSet *R, BParams *P)
{
    for (int i = 0; i < kLanes; ++i) {
        R->r[i] = i < k ? roots[i] : -1;
        if (i < k && roots[i] == g->fail_root) P->fail_injected = 1;
    }
}

// [init, seed, L x (push, pull), finisher, level pass] for one group of at
// most 64 roots.
int enqueue_batch(Graph *g, BatchWorkspace *w, const bfs_options &opt, const int32_t *roots, int k,
                  const LanePtrs &out, hipStream_t s, bool profile, int *layers_enqueued)
{
    BParams P;
    fill_batch_params(g, w, opt, k, &P);
    RootSet R;
    fill_roots(g, roots, k, &R, &P);
    const int grid = opt.grid_blocks > 0 ? opt.grid_blocks : g->batch_grid;
    const int pgrid = opt.grid_blocks > 0 ? opt.grid_blocks : g->batch_pull_grid;
    const int L = opt.layers_per_launch > 0 ? opt.layers_per_launch : g->batch_depth.typical.load();
    hipError_t e;
    if (profile) {
        while ((int)w->layer_ev.size() < 2 * L) {
            hipEvent_t ev;
            if ((e = hipEventCreateWithFlags(&ev, hipEventDisableSystemFence)) != hipSuccess)
                return hip_fail(e, "event");
            w->layer_ev.push_back(ev);
        }
    }
    if ((e = launch_batch_init(P, out, grid, s)) != hipSuccess) return hip_fail(e, "batch init launch");
    if ((e = launch_batch_seed(P, R, s)) != hipSuccess) return hip_fail(e, "batch seed launch");
    for (int i = 0; i < L; ++i) {
        if (profile && (e = hipEventRecord(w->layer_ev[2 * i], s)) != hipSuccess) return hip_fail(e, "event");
        if ((e = launch_batch_push(P, i, grid, s)) != hipSuccess) return hip_fail(e, "batch push launch");
        if ((e = launch_batch_pull(P, i, pgrid, s)) != hipSuccess) return hip_fail(e, "batch pull launch");
        if (profile && (e = hipEventRecord(w->layer_ev[2 * i + 1], s)) != hipSuccess) return hip_fail(e, "event");
    }
    if ((e = launch_batch_finish(P, s)) != hipSuccess) return hip_fail(e, "batch finisher launch");
    if ((e = launch_batch_levels(P, grid, s)) != hipSuccess) return hip_fail(e, "batch level pass launch");
    *layers_enqueued = L;
    return BFS_OK;
}

int enqueue_batch_graph(Graph *g, BatchWorkspace *w, const bfs_options &opt, const int32_t *roots, int k,
                        const LanePtrs &out, hipStream_t s, int *layers_enqueued)
{
    BParams P;
    fill_batch_params(g, w, opt, k, &P);
    RootSet R;
    fill_roots(g, roots, k, &R, &P);
    const int grid = opt.grid_blocks > 0 ? opt.grid_blocks : g->batch_grid;
    const int pgrid = opt.grid_blocks > 0 ? opt.grid_blocks : g->batch_pull_grid;
    const int L = opt.layers_per_launch > 0 ? opt.layers_per_launch : g->batch_depth.typical.load();
    char key[160];
    snprintf(key, sizeof key, "%d/%d/%lld/%lld/%d/%d/%d/%d", k, opt.rule, P.alpha, P.beta, P.wpg, grid, pgrid, L);
    hipError_t e;
    auto it = w->replays.find(key);
    if (it == w->replays.end()) {
        BatchWorkspace::Replay Q;
        Q.grid = grid;
        Q.layers = L;
        // the node arguments are copied when a node is added
        std::vector<int> layer_idx(L);
        for (int i = 0; i < L; ++i) layer_idx[i] = i;
        if ((e = hipGraphCreate(&Q.graph, 0)) != hipSuccess) return hip_fail(e, "graph create");
        hipGraphNode_t prev = nullptr;
        auto add = [&](int which, dim3 gd, dim3 bd, void **args, hipGraphNode_t *keep) -> hipError_t {
            hipKernelNodeParams np;
            std::memset(&np, 0, sizeof np);
            np.func = kernel_ptr_batch(which);
            np.gridDim = gd;
            np.blockDim = bd;
            np.kernelParams = args;
            hipGraphNode_t node;
            const hipError_t r = hipGraphAddKernelNode(&node, Q.graph, prev ? &prev : nullptr, prev ? 1 : 0, &np);
            if (r == hipSuccess) {
                prev = node;
                if (keep) *keep = node;
            }
            return r;
        };
        LanePtrs o = out;
        void *init_args[] = {&P, &o};
        void *seed_args[] = {&P, &R};
        void *fin_args[] = {&P};
        // a graph that could not be built completely is destroyed
        auto fail = [&](hipError_t err, const char *what) {
            hipGraphDestroy(Q.graph);
            return hip_fail(err, what);
        };
        if ((e = add(BK_INIT, dim3(grid, k + 1), dim3(kBlock), init_args, &Q.init)) != hipSuccess ||
            (e = add(BK_SEED, dim3(1), dim3(64), seed_args, &Q.seed)) != hipSuccess)
            return fail(e, "graph batch nodes");
        for (int i = 0; i < L; ++i) {
            void *args[] = {&P, &layer_idx[i]};
            if ((e = add(BK_PUSH, dim3(grid), dim3(kBlock), args, nullptr)) != hipSuccess ||
                (e = add(BK_PULL, dim3(pgrid), dim3(kPullWaves * 64), args, nullptr)) != hipSuccess)
                return fail(e, "graph batch layer nodes");
        }
        if ((e = add(BK_FINISH, dim3(1), dim3(kFinishBlock), fin_args, nullptr)) != hipSuccess ||
            (e = add(BK_LEVELS, dim3(grid), dim3(kBlock), fin_args, nullptr)) != hipSuccess)
            return fail(e, "graph batch finisher nodes");
        if ((e = hipGraphInstantiate(&Q.exec, Q.graph, nullptr, nullptr, 0)) != hipSuccess)
            return fail(e, "graph instantiate");
        it = w->replays.emplace(key, Q).first;
    }
    BatchWorkspace::Replay &Q = it->second;
    // the run's outputs, flags and roots into the two nodes that read them
    LanePtrs o = out;
    void *init_args[] = {&P, &o};
    void *seed_args[] = {&P, &R};
    hipKernelNodeParams kp;
    std::memset(&kp, 0, sizeof kp);
    kp.func = kernel_ptr_batch(BK_INIT);
    kp.gridDim = dim3(Q.grid, k + 1);
    kp.blockDim = dim3(kBlock);
    kp.kernelParams = init_args;
    if ((e = hipGraphExecKernelNodeSetParams(Q.exec, Q.init, &kp)) != hipSuccess) return hip_fail(e, "graph update");
    kp.func = kernel_ptr_batch(BK_SEED);
    kp.gridDim = dim3(1);
    kp.blockDim = dim3(64);
    kp.kernelParams = seed_args;
    if ((e = hipGraphExecKernelNodeSetParams(Q.exec, Q.seed, &kp)) != hipSuccess) return hip_fail(e, "graph update");
    if ((e = hipGraphLaunch(Q.exec, s)) != hipSuccess) return hip_fail(e, "graph launch");
    *layers_enqueued = Q.layers;
    return BFS_OK;
}

}  // namespace hybfs

using namespace hybfs;

extern "C" {

int bfs_run_batch(bfs_graph_t gh, const int32_t *roots, int32_t k, int32_t *level_out, int32_t *parent_out,
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
    if (opt.rule == BFS_RULE_TABLE)
        return set_error(BFS_E_INVALID, "batched runs take the edge rule or a forced direction");
    if (k < 1) return set_error(BFS_E_INVALID, "k = %d roots; need at least one", k);
    if (!roots) return set_error(BFS_E_INVALID, "NULL roots");
    for (int i = 0; i < k; ++i)
        if (roots[i] < 0 || (int64_t)roots[i] >= g->n)
            return set_error(BFS_E_INVALID, "roots[%d] = %d out of [0, %lld)", i, roots[i], (long long)g->n);
    if (!level_out || !parent_out) return set_error(BFS_E_INVALID, "NULL output");
    if (opt.async && (!opt.out_on_device || stats))
        return set_error(BFS_E_INVALID, "async runs need device outputs and no stats");

    BatchWorkspace *w = nullptr;
    rc = get_batch_workspace(g, opt.stream, &w);
    if (rc) return rc;
    std::lock_guard<std::mutex> wl(w->mu);
    hipStream_t s = (hipStream_t)opt.stream;
    hipError_t e;
    const long long n = g->n;
    const int kmax = std::min<int>(k, kLanes);

    int *stage = nullptr;
    if (!opt.out_on_device) {
        const long long need = 2 * (long long)kmax * n;
        if (!w->out_tmp || w->out_tmp_elems < need) {
            if (w->out_tmp) {
                hipStreamSynchronize(s);
                hipFree(w->out_tmp);
                w->out_tmp = nullptr;
            }
            if ((e = hipMalloc(&w->out_tmp, need * 4)) != hipSuccess) return hip_fail(e, "output staging");
            w->out_tmp_elems = need;
        }
        stage = w->out_tmp;
    }

    const bool profile = opt.profile_layers && stats && !opt.async;
    if (stats) {
        stats->num_layers = 0;
        stats->reached = 0;
        stats->reached_degree_sum = 0;
        stats->device_us = 0.0;
        stats->layer_launches = 0;
        stats->layer0_kernel = 0;
        stats->layer_kernel_us = 0.0;
    }
    for (int g0 = 0; g0 < k; g0 += kLanes) {
        const int kg = std::min(kLanes, k - g0);
        int *lvl = opt.out_on_device ? level_out + (long long)g0 * n : stage;
        int *par = opt.out_on_device ? parent_out + (long long)g0 * n : stage + (long long)kg * n;
        int launched = 0;
        if (stats && (e = hipEventRecord(w->e0, s)) != hipSuccess) return hip_fail(e, "event record");
        LanePtrs out;
        for (int b = 0; b < kLanes; ++b) {
            out.level[b] = b < kg ? lvl + (long long)b * n : nullptr;
            out.parent[b] = b < kg ? par + (long long)b * n : nullptr;
        }
        if (opt.graph_launch && !profile) rc = enqueue_batch_graph(g, w, opt, roots + g0, kg, out, s, &launched);
        else rc = enqueue_batch(g, w, opt, roots + g0, kg, out, s, profile, &launched);
        if (rc) return rc;
        if (stats && (e = hipEventRecord(w->e1, s)) != hipSuccess) return hip_fail(e, "event record");
        if (opt.async) continue;

        if ((e = hipMemcpyAsync(w->h_ctrl, w->ctrl, sizeof(BCtrl), hipMemcpyDeviceToHost, s)) != hipSuccess)
            return hip_fail(e, "control copy");
        if (!opt.out_on_device) {
            if ((e = hipMemcpyAsync(level_out + (long long)g0 * n, lvl, (size_t)kg * n * 4, hipMemcpyDeviceToHost,
                                    s)) != hipSuccess ||
                (e = hipMemcpyAsync(parent_out + (long long)g0 * n, par, (size_t)kg * n * 4,
                                    hipMemcpyDeviceToHost, s)) != hipSuccess)
                return hip_fail(e, "copy outputs to host");
        }
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "batched traversal");
        const BCtrl &c = *w->h_ctrl;
        if (c.done != 1 || c.status != 0)
            return set_error(BFS_E_DEVICE, "batched traversal failed a device-side check (done %d, status %d)",
                             c.done, c.status);
        g->batch_depth.note(c.nlayers);
        if (!stats) continue;
        float ms = 0.f;
        hipEventElapsedTime(&ms, w->e0, w->e1);
        stats->device_us += ms * 1000.0;
        stats->num_layers = std::max(stats->num_layers, c.nlayers);
        stats->reached += c.pairs;
        stats->reached_degree_sum += c.pairs_deg;
        stats->layer_launches += 2 * launched;
        std::vector<double> kus(launched, 0.0);
        if (profile) {
            for (int i = 0; i < launched; ++i) {
                float lm = 0.f;
                hipEventElapsedTime(&lm, w->layer_ev[2 * i], w->layer_ev[2 * i + 1]);
                kus[i] = lm * 1000.0;
                stats->layer_kernel_us += kus[i];
            }
        }
        // layer records describe the first group
        const int nrec = std::min(c.nlayers, kTraceCap);
        if (g0 == 0 && stats->layers && stats->capacity > 0 && nrec > 0) {
            const int ncopy = std::min(nrec, stats->capacity);
            e = hipMemcpy(w->h_trace, w->trace, nrec * sizeof(LayerRec), hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_fail(e, "trace copy");
            for (int i = 0; i < ncopy; ++i) {
                const LayerRec &r = w->h_trace[i];
                bfs_layer_stat &o = stats->layers[i];
                o.direction = r.dir;
                o.reserved = 0;
                o.n_f = r.n_f;
                o.m_f = r.m_f;
                o.m_u = r.m_u;
                o.v_u = r.v_u;
                o.kernel_us = (profile && i < launched) ? kus[i] : 0.0;
                o.t_us = o.kernel_us;
                for (int k = 0; k < 6; ++k) o.work[k] = 0;
            }
        }
    }
    return BFS_OK;
}

}  // extern "C"
