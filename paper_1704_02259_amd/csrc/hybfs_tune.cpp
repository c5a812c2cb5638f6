// Autotuner (bfs_autotune): coordinate descent over the traversal options
// that change speed but never results -- the switch parameters of Algorithm
// 3 (alpha, beta), the bottom-up probe depth (MAX_POS, Section 5.2), the
// top-down degree cut-off, the wavefront task size and the grid -- timed with
// HIP events on the caller's roots.
#include <algorithm>
#include <cstring>
#include <vector>

#include "hybfs_internal.h"

namespace hybfs {

namespace {

struct Tuner {
    Graph *g;
    const int32_t *roots;
    int k;
    int mode;
    hipStream_t s;
    int *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int trials = 0;

    ~Tuner()
    {
        if (out) hipFree(out);
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
    }

    int enqueue(const bfs_options &o)
    {
        bfs_graph_t gh = reinterpret_cast<bfs_graph_t>(g);
        if (mode == 0) {
            for (int i = 0; i < k; ++i) {
                const int rc = bfs_run(gh, roots[i], out, out + g->n, &o, nullptr);
                if (rc) return rc;
            }
            return BFS_OK;
        }
        return bfs_run_batch(gh, roots, k, out, out + (long long)k * g->n, &o, nullptr);
    }

    // Time of one pass over the roots with options o (best of two, after an
    // untimed pass that also checks the options and adapts the launch depth).
    int measure(const bfs_options &base, double *us)
    {
        bfs_options o = base;
        o.stream = s;
        o.out_on_device = 1;
        o.async = 0;
        int rc = enqueue(o);
        if (rc) return rc;
        o.async = 1;
        double best = 1e30;
        for (int rep = 0; rep < 2; ++rep) {
            hipError_t e;
            if ((e = hipEventRecord(e0, s)) != hipSuccess) return hip_fail(e, "event");
            if ((rc = enqueue(o))) return rc;
            if ((e = hipEventRecord(e1, s)) != hipSuccess) return hip_fail(e, "event");
            if ((e = hipEventSynchronize(e1)) != hipSuccess) return hip_fail(e, "tuning run");
            float ms = 0.f;
            hipEventElapsedTime(&ms, e0, e1);
            best = std::min(best, (double)ms * 1000.0);
        }
        // the timed passes ran asynchronously: their failures surface here
        if ((rc = check_async_errors(g, (void *)s))) return rc;
        ++trials;
        *us = best;
        return BFS_OK;
    }
};

struct Knob {
    int32_t bfs_options::*field;
    std::vector<int32_t> values;
};

}  // namespace
}  // namespace hybfs

using namespace hybfs;

extern "C" {

int bfs_autotune(bfs_graph_t gh, const int32_t *roots, int32_t k, int32_t mode, int32_t max_trials,
                 bfs_options *opt, bfs_tune_report *report)
{
    clear_error();
    if (!gh || !roots || !opt) return set_error(BFS_E_INVALID, "NULL argument");
    if (k < 1) return set_error(BFS_E_INVALID, "need at least one root");
    if (mode != 0 && mode != 1) return set_error(BFS_E_INVALID, "mode must be 0 (single) or 1 (batch)");
    if (max_trials < 1) return set_error(BFS_E_INVALID, "max_trials must be >= 1");
    Graph *g = reinterpret_cast<Graph *>(gh);
    for (int i = 0; i < k; ++i)
        if (roots[i] < 0 || roots[i] >= g->n) return set_error(BFS_E_INVALID, "roots[%d] out of range", i);
    bfs_options start = *opt;
    start.async = 0;
    start.profile_layers = 0;
    int rc = validate_options(start);
    if (rc) return rc;
    if (mode == 1) {
        if (start.rule == BFS_RULE_TABLE) start.rule = BFS_RULE_EDGES;
        start.graph_launch = 0;
    }

    Tuner T;
    T.g = g;
    T.roots = roots;
    T.k = k;
    T.mode = mode;
    T.s = (hipStream_t)opt->stream;
    hipError_t e;
    const long long outs = mode == 0 ? 2 * g->n : 2LL * k * g->n;
    if ((e = hipMalloc(&T.out, outs * 4)) != hipSuccess) return hip_fail(e, "tuning outputs");
    // timing-only events: no system-scope fence inside the measured window
    if ((e = hipEventCreateWithFlags(&T.e0, hipEventDisableSystemFence)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&T.e1, hipEventDisableSystemFence)) != hipSuccess)
        return hip_fail(e, "event");

    const int grid0 = mode == 0 ? g->grid_default : g->batch_grid;
    std::vector<Knob> knobs = {
        {&bfs_options::alpha, {2, 4, 8, 14, 24, 48, 96, 256}},
        {&bfs_options::beta, {4, 8, 16, 24, 48, 96, 256}},
        {&bfs_options::words_per_wave, {0, 1, 2, 4, 8, 16, 32}},
        {&bfs_options::grid_blocks, {0, std::max(1, grid0 / 4), std::max(1, grid0 / 2), grid0 * 2}},
    };
    if (mode == 0) {
        knobs.push_back({&bfs_options::probe_k, {0, 2, 4, 8, 16, 32}});
        knobs.push_back({&bfs_options::td_hub_degree, {256, 1024, 4096, 16384}});
        knobs.push_back({&bfs_options::bu_serial_probes, {0, 1, -1}});
        if (g->bin_auto) knobs.push_back({&bfs_options::alpha_binned, {0, 2, 4, 6, 8, 14}});
    }

    double best_us = 0.0;
    if ((rc = T.measure(start, &best_us))) return rc;
    const double start_us = best_us;
    bfs_options best = start;
    int rounds = 0;
    bool improved = true;
    while (improved && T.trials < max_trials && rounds < 4) {
        improved = false;
        ++rounds;
        for (const Knob &kn : knobs) {
            for (int32_t v : kn.values) {
                if (T.trials >= max_trials) break;
                if (best.*kn.field == v) continue;
                bfs_options trial = best;
                trial.*kn.field = v;
                double us = 0.0;
                if ((rc = T.measure(trial, &us))) return rc;
                // a new setting must win by 2% to replace the incumbent
                if (us < best_us * 0.98) {
                    best_us = us;
                    best = trial;
                    improved = true;
                }
            }
        }
    }
    best.stream = opt->stream;
    best.out_on_device = opt->out_on_device;
    best.async = opt->async;
    best.profile_layers = opt->profile_layers;
    *opt = best;
    if (report) {
        std::memset(report, 0, sizeof *report);
        report->trials = T.trials;
        report->rounds = rounds;
        report->start_us = start_us;
        report->best_us = best_us;
    }
    return BFS_OK;
}

}  // extern "C"
