// Serving runtime (bfs_serve_*): resident graphs, a request queue per graph,
// and worker slots that each own a HIP stream.  A free slot takes the graph
// whose oldest request has waited longest, drains up to max_batch of its
// queued requests into one traversal (bfs_run for one root, the batched
// multi-source traversal for more), and admits it only when the device
// memory the slots hold after it fits the memory budget.  Requests that
// arrive while others run are picked up by the next free slot (continuous
// batching); slots run concurrently, so their kernels overlap on the device.
//
// Memory accounting: a slot's traversals leave their workspaces cached with
// the graph, keyed by the slot's stream (single-root workspace with its
// binned buckets, queues and output staging; batched workspace), and a slot
// keeps its host-output staging.  All of it is charged to the budget while
// held.  Admission charges what a traversal will add to its slot's holdings;
// when that does not fit, idle holdings are released (the slot's own caches
// of other graphs first, then other idle slots' caches), then a batch is
// halved, then the slot waits for running traversals.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>

#include "hybfs_internal.h"

namespace hybfs {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    int gid = 0;
    int root = 0;
    int *lvl = nullptr, *par = nullptr;
    Clock::time_point t_submit, t_done;
    int state = 0;                 // 0 queued, 1 running, 2 done
    int rc = BFS_OK;
    std::string err;
};

struct WorkerSlot {
    hipStream_t stream = nullptr;
    int *stage = nullptr;          // host-output staging of a batch: level, then parent rows
    long long stage_elems = 0;
    // a traversal runs on this slot; while it does, the slot's worker owns
    // stage and the workspaces, and the slot is charged busy_charge: what it
    // held at admission plus what the traversal may allocate
    bool busy = false;
    long long busy_charge = 0;
    std::map<Graph *, long long> cache;   // device bytes of each graph's workspaces on `stream`
    long long idle_charge() const
    {
        long long u = stage_elems * 4;
        for (const auto &c : cache) u += c.second;
        return u;
    }
};

struct Server {
    bfs_serve_config cfg;
    int dev = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::vector<Graph *> graphs;
    std::vector<std::deque<Request *>> queues;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    uint64_t next_ticket = 1;
    std::vector<WorkerSlot> slots;
    std::vector<std::thread> workers;
    int running_batches = 0;
    bool stopping = false;
    long long used = 0, peak = 0;  // bytes held + reserved by all slots, and its maximum
    // statistics since creation or the last reset
    long long submitted = 0, completed = 0, failed = 0, batches = 0, batched_requests = 0, admission_waits = 0,
              evictions = 0;
    std::vector<double> lat_us;
    double te = 0.0;
    bool have_first = false;
    Clock::time_point first_submit, last_done;
    long long open = 0;            // queued + running
    // per graph: running averages of a single-root traversal and of a batched
    // traversal (host clock around the run); 0 = not measured yet
    std::vector<double> t_single_us, t_batch_us;

    void worker(int i);
    void recount()
    {
        long long u = 0;
        for (const WorkerSlot &sl : slots) u += sl.busy ? sl.busy_charge : sl.idle_charge();
        used = u;
        peak = std::max(peak, used);
    }
    long long need(int i, Graph *g, int k, const bfs_options &opt) const;
    bool evict_one(int i, Graph *g, bool keep_stage);
    int batch_threshold(int gid) const
    {
        if (cfg.batch_threshold > 0) return cfg.batch_threshold;
        const double ts = t_single_us[gid], tb = t_batch_us[gid];
        if (ts <= 0.0) return 2;                  // nothing measured yet: batch what is there
        if (tb <= 0.0) return 16;
        return (int)std::min(64.0, std::max(2.0, std::ceil(tb / ts)));
    }
    int run_group(int i, Graph *g, std::vector<Request *> &rq, double *te_out);
};

// Options of every traversal the server runs (the stream is the slot's).
static bfs_options serve_options(const bfs_serve_config &cfg, hipStream_t s)
{
    bfs_options opt;
    bfs_options_init(&opt);
    if (cfg.alpha > 0) opt.alpha = cfg.alpha;
    if (cfg.beta > 0) opt.beta = cfg.beta;
    opt.stream = s;
    opt.out_on_device = cfg.out_on_device;
    return opt;
}

// Bytes slot i's holdings grow by when it runs k roots of g (lock held).
long long Server::need(int i, Graph *g, int k, const bfs_options &opt) const
{
    const WorkerSlot &sl = slots[i];
    size_t single = 0, batch = 0;
    held_bytes(g, sl.stream, &single, &batch);
    long long after;
    long long stage = sl.stage_elems * 4;
    if (k == 1) {
        after = (long long)single_run_bytes(g, sl.stream, opt) + (long long)batch;
    } else {
        after = (long long)single + (long long)(batch ? batch : batch_workspace_bytes(g));
        // a smaller staging buffer is freed before the larger one is allocated
        if (!cfg.out_on_device) stage = std::max(stage, 8LL * k * g->n);
    }
    auto it = sl.cache.find(g);
    const long long before = it != sl.cache.end() ? it->second : 0;
    return std::max(0LL, after - before) + (stage - sl.stage_elems * 4);
}

// Releases the largest idle holding (lock held; it blocks while the device
// frees): slot i's caches of graphs other than g, its staging unless
// keep_stage, then what other idle slots hold.  False when there is none.
bool Server::evict_one(int i, Graph *g, bool keep_stage)
{
    for (int pass = 0; pass < 2; ++pass) {
        int bs = -1;
        Graph *bg = nullptr;
        long long best = 0;
        for (int j = 0; j < (int)slots.size(); ++j) {
            const WorkerSlot &sl = slots[j];
            if ((pass == 0) != (j == i) || sl.busy) continue;
            for (const auto &c : sl.cache)
                if ((j != i || c.first != g) && c.second > best) {
                    best = c.second;
                    bs = j;
                    bg = c.first;
                }
            if ((j != i || !keep_stage) && sl.stage_elems * 4 > best) {
                best = sl.stage_elems * 4;
                bs = j;
                bg = nullptr;
            }
        }
        if (bs < 0) continue;
        WorkerSlot &sl = slots[bs];
        if (bg) {
            release_workspaces(bg, sl.stream);
            sl.cache.erase(bg);
        } else {
            hipFree(sl.stage);
            sl.stage = nullptr;
            sl.stage_elems = 0;
        }
        ++evictions;
        recount();
        return true;
    }
    return false;
}

// Executes one admitted group on slot i (no lock held).
int Server::run_group(int i, Graph *g, std::vector<Request *> &rq, double *te_out)
{
    WorkerSlot &sl = slots[i];
    hipStream_t s = sl.stream;
    const int k = (int)rq.size();
    const bfs_options opt = serve_options(cfg, s);
    if (k == 1) {
        bfs_stats st;
        std::memset(&st, 0, sizeof st);
        const int rc = bfs_run(reinterpret_cast<bfs_graph_t>(g), rq[0]->root, rq[0]->lvl, rq[0]->par, &opt, &st);
        *te_out = rc == BFS_OK ? st.reached_degree_sum / 2.0 : 0.0;
        return rc;
    }
    BatchWorkspace *w = nullptr;
    int rc = get_batch_workspace(g, s, &w);
    if (rc) return rc;
    std::lock_guard<std::mutex> wl(w->mu);
    const long long n = g->n;
    LanePtrs out;
    std::vector<int32_t> roots(k);
    for (int b = 0; b < kLanes; ++b) {
        out.level[b] = nullptr;
        out.parent[b] = nullptr;
    }
    for (int b = 0; b < k; ++b) {
        roots[b] = rq[b]->root;
        if (cfg.out_on_device) {
            out.level[b] = rq[b]->lvl;
            out.parent[b] = rq[b]->par;
        } else {
            out.level[b] = sl.stage + (long long)b * n;
            out.parent[b] = sl.stage + (long long)(k + b) * n;
        }
    }
    int launched = 0;
    rc = enqueue_batch(g, w, opt, roots.data(), k, out, s, false, &launched);
    if (rc) return rc;
    hipError_t e;
    if ((e = hipMemcpyAsync(w->h_ctrl, w->ctrl, sizeof(BCtrl), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "control copy");
    if (!cfg.out_on_device) {
        for (int b = 0; b < k; ++b) {
            if ((e = hipMemcpyAsync(rq[b]->lvl, out.level[b], n * 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
                (e = hipMemcpyAsync(rq[b]->par, out.parent[b], n * 4, hipMemcpyDeviceToHost, s)) != hipSuccess)
                return hip_fail(e, "copy outputs to host");
        }
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "batched traversal");
    const BCtrl &c = *w->h_ctrl;
    if (c.done != 1 || c.status != 0)
        return set_error(BFS_E_DEVICE, "batched traversal failed a device-side check (done %d, status %d)", c.done,
                         c.status);
    g->batch_depth.note(c.nlayers);
    *te_out = c.pairs_deg / 2.0;
    return BFS_OK;
}

void Server::worker(int i)
{
    // the server's device for this thread; should that fail, every query
    // this slot takes fails with the error instead of running elsewhere
    const hipError_t dev_err = hipSetDevice(dev);
    WorkerSlot &sl = slots[i];
    const bool host_out = !cfg.out_on_device;
    const bfs_options opt = serve_options(cfg, sl.stream);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        // the graph whose head request is oldest
        int gid = -1;
        for (size_t q = 0; q < queues.size(); ++q)
            if (!queues[q].empty() && (gid < 0 || queues[q].front()->t_submit < queues[gid].front()->t_submit))
                gid = (int)q;
        if (gid < 0) {
            if (stopping) break;
            cv_work.wait(lk);
            continue;
        }
        Graph *g = graphs[gid];
        // batch only when the queue is deep enough for one batched traversal
        // to beat that many single ones; otherwise take one query and leave
        // the rest to the other slots
        int k = (int)std::min<size_t>(queues[gid].size(), (size_t)cfg.max_batch);
        if (k > 1 && k < batch_threshold(gid)) k = 1;
        // admission: the slots may hold at most memory_budget; idle caches
        // go first, then the batch shrinks
        long long F = need(i, g, k, opt);
        while (used + F > cfg.memory_budget) {
            if (!evict_one(i, g, k > 1 && host_out)) {
                if (k == 1) break;
                k = std::max(1, k / 2);
            }
            F = need(i, g, k, opt);
        }
        if (used + F > cfg.memory_budget) {
            if (running_batches == 0) {
                // nothing in flight will free memory: this request cannot be served
                Request *r = queues[gid].front();
                queues[gid].pop_front();
                r->state = 2;
                r->rc = BFS_E_NOMEM;
                r->err = "request does not fit the serving memory budget";
                r->t_done = Clock::now();
                ++failed;
                --open;
                cv_done.notify_all();
                continue;
            }
            ++admission_waits;
            cv_done.wait(lk);
            continue;
        }
        std::vector<Request *> rq;
        for (int j = 0; j < k; ++j) {
            rq.push_back(queues[gid].front());
            queues[gid].pop_front();
            rq.back()->state = 1;
        }
        sl.busy_charge = sl.idle_charge() + F;
        sl.busy = true;
        recount();
        ++running_batches;
        ++batches;
        if (k > 1) batched_requests += k;
        lk.unlock();

        int rc = BFS_OK;
        if (k > 1 && host_out && sl.stage_elems < 2LL * k * g->n) {
            if (sl.stage) {
                hipFree(sl.stage);
                sl.stage = nullptr;
                sl.stage_elems = 0;
            }
            const long long want = 2LL * k * g->n;
            if (hipMalloc(&sl.stage, want * 4) != hipSuccess) rc = set_error(BFS_E_NOMEM, "serving output staging");
            else sl.stage_elems = want;
        }
        double te_group = 0.0;
        const Clock::time_point t_start = Clock::now();
        if (rc == BFS_OK && dev_err != hipSuccess) rc = hip_fail(dev_err, "serving worker device");
        if (rc == BFS_OK) rc = run_group(i, g, rq, &te_group);
        const double run_us = std::chrono::duration<double, std::micro>(Clock::now() - t_start).count();
        const std::string err = rc != BFS_OK ? std::string(last_error()) : std::string();
        const Clock::time_point t = Clock::now();

        lk.lock();
        sl.busy = false;
        sl.cache[g] = (long long)held_bytes(g, sl.stream, nullptr, nullptr);
        recount();
        --running_batches;
        for (Request *r : rq) {
            r->state = 2;
            r->rc = rc;
            r->err = err;
            r->t_done = t;
            --open;
            if (rc == BFS_OK) {
                ++completed;
                lat_us.push_back(std::chrono::duration<double, std::micro>(t - r->t_submit).count());
            } else {
                ++failed;
            }
        }
        if (rc == BFS_OK) {
            te += te_group;
            last_done = t;
            double &avg = k == 1 ? t_single_us[gid] : t_batch_us[gid];
            avg = avg == 0.0 ? run_us : 0.8 * avg + 0.2 * run_us;
        }
        cv_done.notify_all();
    }
}

}  // namespace hybfs

using namespace hybfs;

extern "C" {

void bfs_serve_config_init(bfs_serve_config *cfg)
{
    if (!cfg) return;
    std::memset(cfg, 0, sizeof *cfg);
    cfg->memory_budget = 0;
    cfg->max_batch = 64;
    cfg->streams = 4;
    cfg->queue_capacity = 65536;
    cfg->out_on_device = 1;
}

int bfs_serve_create(const bfs_serve_config *cfg_in, bfs_server_t *out)
{
    clear_error();
    if (!out) return set_error(BFS_E_INVALID, "NULL output");
    bfs_serve_config cfg;
    if (cfg_in) cfg = *cfg_in;
    else bfs_serve_config_init(&cfg);
    if (cfg.max_batch < 1 || cfg.max_batch > 64) return set_error(BFS_E_INVALID, "max_batch must be in [1, 64]");
    if (cfg.streams < 1 || cfg.streams > 16) return set_error(BFS_E_INVALID, "streams must be in [1, 16]");
    if (cfg.queue_capacity < 1) return set_error(BFS_E_INVALID, "queue_capacity must be >= 1");
    if (cfg.out_on_device < 0 || cfg.out_on_device > 1) return set_error(BFS_E_INVALID, "out_on_device is 0 or 1");
    if (cfg.memory_budget < 0 || cfg.alpha < 0 || cfg.beta < 0)
        return set_error(BFS_E_INVALID, "negative memory_budget, alpha or beta");
    if (cfg.batch_threshold < 0 || cfg.batch_threshold > 64)
        return set_error(BFS_E_INVALID, "batch_threshold must be in [0, 64]");
    std::unique_ptr<Server> S(new (std::nothrow) Server());
    if (!S) return set_error(BFS_E_NOMEM, "host allocation");
    hipError_t e;
    if ((e = hipGetDevice(&S->dev)) != hipSuccess) return hip_fail(e, "current device");
    if (cfg.memory_budget == 0) {
        size_t fr = 0, tot = 0;
        if ((e = hipMemGetInfo(&fr, &tot)) != hipSuccess) return hip_fail(e, "device memory query");
        cfg.memory_budget = (int64_t)(fr / 4 * 3);
    }
    S->cfg = cfg;
    S->slots.resize(cfg.streams);
    for (auto &sl : S->slots)
        if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e, "stream");
    Server *raw = S.get();
    for (int i = 0; i < cfg.streams; ++i) S->workers.emplace_back([raw, i] { raw->worker(i); });
    *out = reinterpret_cast<bfs_server_t>(S.release());
    return BFS_OK;
}

int bfs_serve_add_graph(bfs_server_t sh, bfs_graph_t g, int32_t *graph_id)
{
    clear_error();
    if (!sh || !g || !graph_id) return set_error(BFS_E_INVALID, "NULL argument");
    Server *S = reinterpret_cast<Server *>(sh);
    std::lock_guard<std::mutex> lk(S->mu);
    S->graphs.push_back(reinterpret_cast<Graph *>(g));
    S->queues.emplace_back();
    S->t_single_us.push_back(0.0);
    S->t_batch_us.push_back(0.0);
    *graph_id = (int32_t)S->graphs.size() - 1;
    return BFS_OK;
}

int bfs_serve_submit(bfs_server_t sh, int32_t graph_id, int32_t root, int32_t *level_out, int32_t *parent_out,
                     uint64_t *ticket)
{
    clear_error();
    if (!sh || !ticket || !level_out || !parent_out) return set_error(BFS_E_INVALID, "NULL argument");
    Server *S = reinterpret_cast<Server *>(sh);
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stopping) return set_error(BFS_E_INVALID, "server is shutting down");
    if (graph_id < 0 || graph_id >= (int32_t)S->graphs.size())
        return set_error(BFS_E_NOTFOUND, "unknown graph id %d", graph_id);
    Graph *g = S->graphs[graph_id];
    if (root < 0 || root >= g->n) return set_error(BFS_E_INVALID, "root %d out of [0, %lld)", root, (long long)g->n);
    if (S->open >= S->cfg.queue_capacity) return set_error(BFS_E_BUSY, "queue full (%d requests)", S->cfg.queue_capacity);
    std::unique_ptr<Request> r(new Request());
    r->ticket = S->next_ticket++;
    r->gid = graph_id;
    r->root = root;
    r->lvl = level_out;
    r->par = parent_out;
    r->t_submit = Clock::now();
    if (!S->have_first) {
        S->have_first = true;
        S->first_submit = r->t_submit;
    }
    ++S->submitted;
    ++S->open;
    S->queues[graph_id].push_back(r.get());
    *ticket = r->ticket;
    S->reqs.emplace(r->ticket, std::move(r));
    S->cv_work.notify_one();
    return BFS_OK;
}

// Completion of a finished request: releases the ticket and returns its status.
static int release(Server *S, std::unordered_map<uint64_t, std::unique_ptr<Request>>::iterator it)
{
    const int rc = it->second->rc;
    std::string err = it->second->err;
    S->reqs.erase(it);
    if (rc != BFS_OK) return set_error(rc, "%s", err.c_str());
    return BFS_OK;
}

int bfs_serve_poll(bfs_server_t sh, uint64_t ticket, int32_t *done)
{
    clear_error();
    if (!sh || !done) return set_error(BFS_E_INVALID, "NULL argument");
    Server *S = reinterpret_cast<Server *>(sh);
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return set_error(BFS_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    *done = it->second->state == 2;
    if (!*done) return BFS_OK;
    return release(S, it);
}

int bfs_serve_wait(bfs_server_t sh, uint64_t ticket, int64_t timeout_us)
{
    clear_error();
    if (!sh) return set_error(BFS_E_INVALID, "NULL server");
    Server *S = reinterpret_cast<Server *>(sh);
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return set_error(BFS_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second.get();
    auto ready = [r] { return r->state == 2; };
    if (timeout_us < 0) {
        S->cv_done.wait(lk, ready);
    } else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
        return set_error(BFS_E_TIMEOUT, "ticket %llu not done after %lld us", (unsigned long long)ticket,
                         (long long)timeout_us);
    }
    return release(S, S->reqs.find(ticket));
}

int bfs_serve_stats(bfs_server_t sh, bfs_serve_report *out)
{
    clear_error();
    if (!sh || !out) return set_error(BFS_E_INVALID, "NULL argument");
    Server *S = reinterpret_cast<Server *>(sh);
    std::lock_guard<std::mutex> lk(S->mu);
    std::memset(out, 0, sizeof *out);
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->failed = S->failed;
    long long queued = 0;
    for (auto &q : S->queues) queued += (long long)q.size();
    out->queued = queued;
    out->running = S->open - queued;
    out->batches = S->batches;
    out->batched_requests = S->batched_requests;
    out->admission_waits = S->admission_waits;
    out->evictions = S->evictions;
    out->bytes_in_use = S->used;
    out->peak_bytes = S->peak;
    out->memory_budget = S->cfg.memory_budget;
    if (!S->lat_us.empty()) {
        std::vector<double> l = S->lat_us;
        std::sort(l.begin(), l.end());
        auto pct = [&l](double p) {
            const size_t i = (size_t)std::min<double>((double)l.size() - 1, std::ceil(p * l.size()) - 1);
            return l[i];
        };
        out->p50_us = pct(0.50);
        out->p99_us = pct(0.99);
        double sum = 0;
        for (double x : l) sum += x;
        out->mean_us = sum / l.size();
        out->max_us = l.back();
    }
    out->traversed_edges = S->te;
    if (S->have_first && S->completed > 0) {
        const double sec = std::chrono::duration<double>(S->last_done - S->first_submit).count();
        out->gteps = sec > 0 ? S->te / sec / 1e9 : 0.0;
    }
    return BFS_OK;
}

int bfs_serve_reset_stats(bfs_server_t sh)
{
    clear_error();
    if (!sh) return set_error(BFS_E_INVALID, "NULL server");
    Server *S = reinterpret_cast<Server *>(sh);
    std::lock_guard<std::mutex> lk(S->mu);
    S->submitted = S->completed = S->failed = S->batches = S->batched_requests = S->admission_waits =
        S->evictions = 0;
    S->lat_us.clear();
    S->te = 0.0;
    S->have_first = false;
    S->peak = S->used;
    return BFS_OK;
}

int bfs_serve_destroy(bfs_server_t sh)
{
    clear_error();
    if (!sh) return set_error(BFS_E_INVALID, "NULL server");
    Server *S = reinterpret_cast<Server *>(sh);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
    }
    S->cv_work.notify_all();
    S->cv_done.notify_all();
    for (auto &t : S->workers) t.join();
    for (auto &sl : S->slots) {
        if (sl.stream) hipStreamSynchronize(sl.stream);
        if (sl.stage) hipFree(sl.stage);
        // the workspaces this slot's traversals left with the graphs
        for (Graph *g : S->graphs) release_workspaces(g, sl.stream);
        if (sl.stream) hipStreamDestroy(sl.stream);
    }
    delete S;
    return BFS_OK;
}

}  // extern "C"
