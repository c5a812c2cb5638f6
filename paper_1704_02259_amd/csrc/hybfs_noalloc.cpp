// bfs_run_noalloc: the single-root traversal of bfs_run with its per-traversal
// device memory (visited bitmap, the three rotating frontier bitmaps, the
// control block and the layer trace) in a file-scope device array instead of
// a workspace the library allocates.  For callers that cannot allocate device
// memory.  The kernels are bfs_run's own; only where their scratch lives
// differs, and the binned top-down step (whose buckets would need an
// allocation) is not used, which changes no result.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "../../include/hybfs.h"
#include "bfs_device.h"
#include "hybfs_internal.h"

namespace hybfs {

namespace {

constexpr long long kNoAllocMaxWords = BFS_NOALLOC_MAX_VERTICES / 64;
constexpr size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kVisOff = 0;
constexpr size_t kBmOff = al256((size_t)kNoAllocMaxWords * 8);
constexpr size_t kCtrlOff = kBmOff + al256((size_t)kNoAllocMaxWords * 8 * 3);
constexpr size_t kTraceOff = kCtrlOff + al256(sizeof(Ctrl));
constexpr size_t kFiltOff = kTraceOff + al256((size_t)kTraceCap * sizeof(LayerRec));
constexpr size_t kScratchBytes = kFiltOff + al256((size_t)3 * kFilterWords * 4);
constexpr int kMaxDevices = 64;

}  // namespace

// The scratch array.  Every device the library is loaded on holds its own copy
// until the process ends.  In host code its name is not a device address:
// host code only ever uses the address hipGetSymbolAddress returns for the
// current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

struct NoAllocDevice {
    std::mutex mu;                // calls on one device run one at a time
    bool ready = false;
    unsigned char *ptr = nullptr; // device address of `scratch` on this device
    Workspace ws;                 // views into ptr; owns nothing
};

NoAllocDevice g_noalloc[kMaxDevices];

// Once per device, with that device current: the array's device address and
// a cleared control block (so every counter slot starts at zero).
int noalloc_setup(NoAllocDevice &D, hipStream_t s)
{
    if (D.ready) return BFS_OK;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return set_error(BFS_E_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    unsigned char *b = (unsigned char *)p;
    Workspace &w = D.ws;
    w.vis = (unsigned long long *)(b + kVisOff);
    w.bm = (unsigned long long *)(b + kBmOff);
    w.ctrl = (Ctrl *)(b + kCtrlOff);
    w.trace = (LayerRec *)(b + kTraceOff);
    w.filt = (unsigned *)(b + kFiltOff);
    w.bytes = kScratchBytes;
    w.no_alloc = true;   // no frontier queues or hub lists either
    if ((e = hipMemsetAsync(w.ctrl, 0, sizeof(Ctrl), s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "clearing the scratch control block");
    w.counters_zero = true;
    D.ptr = b;
    D.ready = true;
    return BFS_OK;
}

}  // namespace
}  // namespace hybfs

using namespace hybfs;

extern "C" int bfs_run_noalloc(bfs_graph_t gh, int32_t root, int32_t *level_out, int32_t *parent_out,
                               const bfs_options *opt_in, bfs_stats *stats)
{
    clear_error();
    if (!gh) return set_error(BFS_E_INVALID, "NULL graph");
    Graph *g = reinterpret_cast<Graph *>(gh);
    bfs_options opt;
    if (opt_in) opt = *opt_in;
    else {
        bfs_options_init(&opt);
        opt.out_on_device = 1;
    }
    int rc = validate_options(opt);
    if (rc) return rc;
    if (!opt.out_on_device)
        return set_error(BFS_E_INVALID, "bfs_run_noalloc needs device outputs (out_on_device = 1)");
    if (opt.async || opt.profile_layers || opt.graph_launch)
        return set_error(BFS_E_INVALID, "bfs_run_noalloc runs synchronously, without profile_layers "
                                        "or graph_launch");
    if (g->n > BFS_NOALLOC_MAX_VERTICES)
        return set_error(BFS_E_INVALID, "graph of %lld vertices exceeds the no-allocation limit of %lld",
                         (long long)g->n, (long long)BFS_NOALLOC_MAX_VERTICES);
    if (root < 0 || (int64_t)root >= g->n)
        return set_error(BFS_E_INVALID, "root %d out of [0, %lld)", root, (long long)g->n);
    if (!level_out || !parent_out) return set_error(BFS_E_INVALID, "NULL output");
    if (g->dev < 0 || g->dev >= kMaxDevices) return set_error(BFS_E_INVALID, "device %d out of range", g->dev);
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != g->dev)
        return set_error(BFS_E_INVALID, "the graph lives on device %d but device %d is current", g->dev, cur);

    NoAllocDevice &D = g_noalloc[g->dev];
    std::lock_guard<std::mutex> lk(D.mu);
    hipStream_t s = (hipStream_t)opt.stream;
    if ((rc = noalloc_setup(D, s))) return rc;
    Workspace &w = D.ws;

    // the buckets of the binned top-down step would be an allocation
    opt.td_binned = -1;
    int launched = 0, layer0 = 0;
    rc = enqueue_traversal(g, &w, opt, root, level_out, parent_out, s, &launched, false, &layer0);
    if (rc) return rc;
    Ctrl c;
    if ((e = hipMemcpyAsync(&c, w.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "control copy");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "traversal");
    if (c.done != 1 || c.status != 0)
        return set_error(BFS_E_DEVICE, "traversal failed a device-side check (done %d, status %d)", c.done,
                         c.status);
    g->depth.note(c.nlayers);
    if (stats) {
        stats->num_layers = c.nlayers;
        stats->reached = c.reached;
        stats->reached_degree_sum = c.reached_deg;
        stats->device_us = 0.0;
        stats->layer_launches = launched;
        stats->layer0_kernel = layer0;
        stats->layer_kernel_us = 0.0;
        const int nrec = std::min(std::min(c.nlayers, kTraceCap), std::max(stats->capacity, 0));
        if (stats->layers && nrec > 0) {
            // through a small host buffer, 64 records at a time
            LayerRec buf[64];
            for (int i0 = 0; i0 < nrec; i0 += 64) {
                const int m = std::min(64, nrec - i0);
                if ((e = hipMemcpyAsync(buf, w.trace + i0, m * sizeof(LayerRec), hipMemcpyDeviceToHost, s)) !=
                        hipSuccess ||
                    (e = hipStreamSynchronize(s)) != hipSuccess)
                    return hip_fail(e, "trace copy");
                for (int i = 0; i < m; ++i) {
                    const LayerRec &r = buf[i];
                    bfs_layer_stat &o = stats->layers[i0 + i];
                    o.direction = r.dir;
                    o.reserved = 0;
                    o.n_f = r.n_f;
                    o.m_f = r.m_f;
                    o.m_u = r.m_u;
                    o.v_u = r.v_u;
                    o.kernel_us = 0.0;
                    o.t_us = 0.0;
                    for (int k = 0; k < 6; ++k) o.work[k] = 0;
                }
            }
        }
    }
    return BFS_OK;
}
