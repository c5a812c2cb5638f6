// gfx950 kernels of the hybrid BFS.  A traversal is one init kernel followed
// by one kernel per layer (Algorithm 3's loop body): every block of the layer
// kernel reads the counters of the current frontier, takes the same
// direction decision, and runs either the top-down expansion (Algorithm 1) or
// the bottom-up step (Algorithm 2 with the multiple-parents probes of
// Algorithms 4-5).  Kernel boundaries order the layers; there is no grid-wide
// barrier and no co-residency requirement.  For a root of small degree the
// init kernel also runs layer 0 (each block takes the root's neighbours in
// its own vertex range).  A single-block finisher runs any layers left after
// the enqueued layer kernels (very deep graphs) and clears the counters.
//
// Device memory per traversal:
//   vis      uint64 [W]  bit v&63 of word v>>6: v is in a finished layer, or has
//                        degree 0, or v >= n (bottom-up never looks at it)
//   bm       uint64 [3W] frontier F_d, next frontier F_{d+1}, and a spare that
//                        is cleared during layer d; they rotate with d % 3
//   level, parent int32 [n] written in place (-1 for unreached)
//
// Canonical parents: the smallest-id neighbour one layer up.  Bottom-up finds
// it as the first frontier vertex in a sorted row; top-down takes an unsigned
// atomicMin over every frontier edge into a newly reached vertex.
//
// Ownership: during a layer the wavefront that handles bitmap word w is the
// only writer of vis[w] (and, bottom-up, of next[w] and of level/parent of
// w's 64 vertices), so those writes are plain stores.
#include "bfs_device.h"
#include "bfs_wave.h"

namespace hybfs {

// Direction for layer d from its counters (Algorithm 3 as a state machine).
__device__ __forceinline__ int decide(const Params &P, int cur, long long n_f, long long m_f,
                                      long long m_u, long long v_u)
{
    switch (P.rule) {
    case RULE_TOPDOWN: return DIR_TD;
    case RULE_BOTTOMUP: return DIR_BU;
    case RULE_TABLE: {
        const long long f = v_u / 1024, g = P.n / 64;
        if (cur == DIR_TD && n_f > f) return DIR_BU;
        if (cur == DIR_BU && n_f < g) return DIR_TD;
        return cur;
    }
    default:
        if (cur == DIR_TD && m_f * P.alpha > m_u) return DIR_BU;
        if (cur == DIR_BU && n_f * P.beta < P.n) return DIR_TD;
        return cur;
    }
}

// ---------------------------------------------------------------------------
// Lists of the next frontier F_{d+1}.  Every helper here runs with all lanes
// of the wavefront active; a lane without an entry passes false.

// Algorithm 1's out.add, aggregated per wavefront: one atomic on the queue's
// tail reserves the entries of the whole wavefront (ballot + popcount), and
// each lane writes at the count of entries of the lanes below it (mbcnt).
__device__ __forceinline__ void queue_append1(const Params &P, int d, bool f, int v)
{
    const unsigned long long m = __ballot(f);
    if (!m) return;
    unsigned long long base = 0;
    if (__lane_id() == 0)
        base = atomicAdd(&P.ctrl->slot[(d + 1) % kSlots].c[0][kQueueTail], (unsigned long long)__popcll(m));
    base = bcast_u64(base, 0);
    const long long pos =
        (long long)base + __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
    if (f) {
        if (pos < P.q_cap) queue_of(P, d + 1)[pos] = v;
        else atomicOr((unsigned *)&P.ctrl->status, 0x400u);
    }
}

// The same for up to four entries per lane (entry q of every lane, q = 0..3):
// one atomic for the wavefront's total; entry q of a lane goes after all
// entries of index < q and after entry q of the lanes below it.  Only scalar
// prefix sums and one mbcnt per entry, so it adds few vector registers to
// the edge loop it runs in.
__device__ __forceinline__ void queue_append4(const Params &P, int d, const bool (&f)[4], const int (&v)[4])
{
    unsigned long long m[4];
    int pre[4];
    int total = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        m[q] = __ballot(f[q]);
        pre[q] = total;
        total += __popcll(m[q]);
    }
    if (total == 0) return;
    unsigned long long base = 0;
    if (__lane_id() == 0)
        base = atomicAdd(&P.ctrl->slot[(d + 1) % kSlots].c[0][kQueueTail], (unsigned long long)total);
    base = bcast_u64(base, 0);
    int *dst = queue_of(P, d + 1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (f[q]) {
            const long long pos = (long long)base + pre[q] +
                                  __builtin_amdgcn_mbcnt_hi((unsigned)(m[q] >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((unsigned)m[q], 0u));
            if (pos < P.q_cap) dst[pos] = v[q];
            else atomicOr((unsigned *)&P.ctrl->status, 0x400u);
        }
    }
}

// Bitmap-to-queue conversion of a wavefront task's output words: lane l holds
// the found-vertex word wbase + l (0 past the task).  Popcount, prefix sum,
// one atomic for the task's total, then each lane scatters its word's
// vertices in ascending order, so the task's vertices land ascending.
__device__ __forceinline__ void queue_append_words(const Params &P, int d, long long wbase, unsigned long long wm)
{
    const int lane = __lane_id();
    const int c = __popcll(wm);
    const int incl = wave_incl_scan32(c);
    const int total = __builtin_amdgcn_readlane(incl, 63);
    if (total == 0) return;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(&P.ctrl->slot[(d + 1) % kSlots].c[0][kQueueTail], (unsigned long long)total);
    base = bcast_u64(base, 0);
    long long pos = (long long)base + incl - c;
    int *dst = queue_of(P, d + 1);
    const long long v0 = (wbase + lane) << 6;
    while (wm) {
        const int b = __ffsll((long long)wm) - 1;
        wm &= wm - 1;
        if (pos < P.q_cap) dst[pos] = (int)(v0 + b);
        else atomicOr((unsigned *)&P.ctrl->status, 0x400u);
        ++pos;
    }
}

// Where a step appends the hubs it discovers: F_{d+1}'s hub list.
struct HubSink {
    const int *deg;
    unsigned long long *tail;
    Item *dst;
    long long cap;
    unsigned *status;
    int chunk_log2;
};

__device__ __forceinline__ HubSink hub_sink(const Params &P, int d)
{
    return HubSink{P.deg, &P.ctrl->slot[(d + 1) % kSlots].c[0][kHubTail], hubs_of(P, d + 1), P.hq_cap,
                   (unsigned *)&P.ctrl->status, P.chunk_log2};
}

// Hubs discovered inside the edge and probe loops are staged in LDS (one
// LDS atomic per hub, almost no registers in those loops) and written to the
// hub list by the whole block once the step is done (hub_flush), with one
// device atomic per block: appends to one global tail serialise, so they are
// aggregated as far up as the kernel allows.
//
// A list pays only while it is short: a top-down layer whose frontier holds
// many hubs reads most of the hub table anyway, and such a frontier is
// usually followed by a bottom-up layer that does not read the list at all.
// So a list longer than a quarter of the table (all of it for tables under
// 16384 entries) is abandoned: a block that
// stages more than kHubStage hubs, or finds the tail already past that
// limit, only pushes the tail past it, and the consumer then falls back to
// the table (hub_list_usable).
constexpr int kHubStage = 256;
struct HubStage {
    int n;                           // hubs staged (may exceed kHubStage: abandoned)
    int tot;                         // their chunks
    int cur;                         // chunks placed so far
    int pad;
    unsigned long long base;         // the block's range of the hub list
    int v[kHubStage];
};

// Longest hub list worth keeping (entries).
__device__ __forceinline__ long long hub_list_limit(const Params &P)
{
    return P.hq_cap >= 16384 ? P.hq_cap >> 2 : P.hq_cap;
}

__device__ __forceinline__ bool hub_list_usable(const Params &P, long long len)
{
    return len <= hub_list_limit(P);
}

__device__ __forceinline__ void hub_stage_reset(HubStage *hs)
{
    hs->n = 0;
    hs->tot = 0;
    hs->cur = 0;
}

__device__ __forceinline__ int hub_chunks(const HubSink &S, int v)
{
    const long long du = S.deg[v];
    return (int)((du + (1ll << S.chunk_log2) - 1) >> S.chunk_log2);
}

__device__ __forceinline__ void hub_stage(HubStage *hs, int v)
{
    const int i = atomicAdd(&hs->n, 1);
    if (i < kHubStage) hs->v[i] = v;
}

// The block's staged hubs to F_{d+1}'s hub list: their chunks are counted
// in LDS, one device atomic reserves the block's range, and each wavefront
// writes the chunks of the hubs it takes.  The stage is empty afterwards.
// Every thread of the block calls it (it has block barriers).
__device__ __forceinline__ void hub_flush(const Params &P, HubStage *hs, int d, int nwaves_block)
{
    __syncthreads();
    const int n = hs->n;
    if (n > 0) {
        const HubSink S = hub_sink(P, d);
        const long long limit = hub_list_limit(P);
        const int lane = __lane_id();
        if (n <= kHubStage)
            for (int i = threadIdx.x; i < n; i += nwaves_block * 64) atomicAdd(&hs->tot, hub_chunks(S, hs->v[i]));
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long b = ~0ull;
            const long long seen = (long long)__hip_atomic_load(S.tail, __ATOMIC_RELAXED, AGENT);
            if (n > kHubStage || seen > limit) {
                // abandoned: make sure the tail ends past the limit
                if (seen <= limit) atomicAdd(S.tail, (unsigned long long)(limit + 1));
            } else {
                b = atomicAdd(S.tail, (unsigned long long)hs->tot);
                if ((long long)b + hs->tot > limit) b = ~0ull;
            }
            hs->base = b;
        }
        __syncthreads();
        const unsigned long long base = hs->base;
        if (base != ~0ull) {
            for (int i = threadIdx.x >> 6; i < n; i += nwaves_block) {
                const int u = hs->v[i];
                const int nk = hub_chunks(S, u);
                int off = 0;
                if (lane == 0) off = atomicAdd(&hs->cur, nk);
                off = __builtin_amdgcn_readlane(off, 0);
                for (int c = lane; c < nk; c += 64) S.dst[base + off + c] = Item{u, c};
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) hub_stage_reset(hs);
}

// ---------------------------------------------------------------------------
// Membership filter of a small frontier (a Bloom filter with two hashes over
// 2^kFilterLog2 bits).  A bottom-up layer after a small top-down layer probes
// mostly non-members: the filter, copied into LDS, answers most of them
// without touching the frontier bitmap, which at 2^26 vertices does not fit
// in the L2.  Members always pass; a pass is confirmed with the bitmap.
__device__ __forceinline__ unsigned filt_h1(int v) { return (unsigned)v & ((1u << kFilterLog2) - 1u); }
__device__ __forceinline__ unsigned filt_h2(int v) { return ((unsigned)v * 2654435761u) >> (32 - kFilterLog2); }

__device__ __forceinline__ unsigned *filt_of(const Params &P, int d) { return P.filt + (d % 3) * kFilterWords; }

__device__ __forceinline__ void filter_set(unsigned *f, int v)
{
    const unsigned a = filt_h1(v), b = filt_h2(v);
    atomicOr(&f[a >> 5], 1u << (a & 31));
    atomicOr(&f[b >> 5], 1u << (b & 31));
}

// Frontier test of a bottom-up probe: the LDS filter first when there is one.
__device__ __forceinline__ bool probe_front(const unsigned long long *front, const unsigned *lf, int u)
{
    if (lf) {
        const unsigned a = filt_h1(u), b = filt_h2(u);
        if (!((lf[a >> 5] >> (a & 31)) & (lf[b >> 5] >> (b & 31)) & 1u)) return false;
    }
    return test_bit(front, u);
}

// ---------------------------------------------------------------------------
// Up to four frontier edges (u_q -> col[j_q]) per lane of a top-down layer.
// A target v is a candidate when it is in no layer <= d (neither in vis nor
// in the frontier).  Canonical parent = the minimum frontier neighbour: a plain
// read of parent[v] skips the atomic when a smaller neighbour already won, and
// the edge whose unsigned atomicMin replaces the initial -1 discovers v.  The
// loads of the four edges are issued together to overlap their latency.
__device__ __forceinline__ void td_edges4(const Params &P, int d, const int (&uq)[4],
                                          const long long (&jq)[4], const bool (&okq)[4],
                                          const unsigned long long *front, unsigned long long *next,
                                          unsigned long long &nf, unsigned long long &mf,
                                          unsigned long long &nh, HubStage *hs, WorkCount &wc)
{
    int v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        bool ok = okq[q];
        if (ok && (unsigned long long)jq[q] >= (unsigned long long)P.nnz) {
            // an edge index outside the CSR would be a kernel bug: report it
            atomicOr((unsigned *)&P.ctrl->status, 4u);
            ok = false;
        }
        v[q] = ok ? P.col[jq[q]] : -1;
    }
    bool cand[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        cand[q] = false;
        if (v[q] >= 0) {
            const int w = v[q] >> 6;
            cand[q] = !(((P.vis[w] | front[w]) >> (v[q] & 63)) & 1ull);
        }
        if (P.count) {
            wc.c[0] += v[q] >= 0;
            wc.c[1] += cand[q];
        }
    }
    if (P.first_writer) {
        // the edge whose atomic OR sets v's next-frontier bit discovers v and
        // writes its parent (a plain read of the word first skips the atomic
        // when another edge already did)
        unsigned long long nw[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) nw[q] = cand[q] ? next[v[q] >> 6] : 0ull;
        unsigned long long ob[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const unsigned long long bit = 1ull << (v[q] & 63);
            cand[q] = cand[q] && !(nw[q] & bit);
            ob[q] = cand[q] ? atomicOr(&next[v[q] >> 6], bit) : 0ull;
            if (P.count) wc.c[2] += cand[q];
        }
        bool win[4];
        int dvq[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            win[q] = cand[q] && !((ob[q] >> (v[q] & 63)) & 1ull);
            dvq[q] = 0;
            if (win[q]) {
                P.level[v[q]] = d + 1;
                P.parent[v[q]] = uq[q];
                nf += 1;
                dvq[q] = P.deg[v[q]];
                mf += (unsigned long long)dvq[q];
                nh += dvq[q] > P.hub_deg;
                if (P.h_write && dvq[q] > P.hub_deg) hub_stage(hs, v[q]);
                if (P.f_write) filter_set(filt_of(P, d + 1), v[q]);
                if (P.count) wc.c[3] += 1;
            }
        }
        if (P.q_write) queue_append4(P, d, win, v);
        return;
    }
    unsigned pv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) pv[q] = cand[q] ? (unsigned)P.parent[v[q]] : 0u;
    unsigned old[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        cand[q] = cand[q] && (unsigned)uq[q] < pv[q];
        old[q] = cand[q] ? atomicMin((unsigned int *)&P.parent[v[q]], (unsigned int)uq[q]) : 0u;
        if (P.count) wc.c[2] += cand[q];
    }
    bool win[4];
    int dvq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        win[q] = cand[q] && old[q] == 0xFFFFFFFFu;
        dvq[q] = 0;
        if (win[q]) {
            P.level[v[q]] = d + 1;
            atomicOr(&next[v[q] >> 6], 1ull << (v[q] & 63));
            nf += 1;
            dvq[q] = P.deg[v[q]];
            mf += (unsigned long long)dvq[q];
            nh += dvq[q] > P.hub_deg;
            if (P.h_write && dvq[q] > P.hub_deg) hub_stage(hs, v[q]);
            if (P.f_write) filter_set(filt_of(P, d + 1), v[q]);
            if (P.count) wc.c[3] += 1;
        }
    }
    if (P.q_write) queue_append4(P, d, win, v);
}

// Where a top-down layer finds its frontier F_d: the bitmap (scanned) or the
// queue the layer before wrote; and F_d's vertices above hub_deg: the list of
// their chunks the layer before wrote, or the graph's whole table of hub
// chunks, each tested against the frontier bitmap.
struct FrontSrc {
    const int *q;          // F_d as a queue, or nullptr: scan the bitmap
    long long qlen;
    bool q_fold;           // queue entries still have to join vis
    const Item *hubs;      // hub chunks to look at
    long long nhubs;       // their number (0: no hub in the frontier)
    bool hubs_listed;      // `hubs` lists only frontier hubs
};

// The edges of the lanes' vertices (u, degree dl, row start sl; dl = 0 for no
// vertex) laid end to end (prefix sum of degrees + shuffle binary search) and
// handed to the sink 256 per round, four per lane.
template <class Sink>
__device__ __forceinline__ void td_expand(const Params &P, int u, int dl, long long sl, Sink &sink)
{
    const int lane = __lane_id();
    const int incl = wave_incl_scan32(dl);
    const int ex = incl - dl;
    const int E = __builtin_amdgcn_readlane(incl, 63);
    for (int r0 = 0; r0 < E; r0 += 256) {
        int uq[4];
        long long jq[4];
        bool okq[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = r0 + q * 64 + lane;
            okq[q] = idx < E;
            const int lo = lane_search(ex, idx);
            uq[q] = __shfl(u, lo);
            jq[q] = __shfl(sl, lo) + (idx - __shfl(ex, lo));
        }
        sink(uq, jq, okq);
    }
}

// Top-down edge enumeration (Algorithm 1's two loops).
//  * From the bitmap: a wavefront task covers G bitmap words.  The task's
//    frontier vertices are laid out over the lanes (64 per round, found by a
//    prefix sum of the words' popcounts and a select of the set bit): the
//    bitmap-to-queue conversion of the frontier, done per wavefront in
//    registers.
//  * From a queue: a task is E <= 64 consecutive entries, E sized so that the
//    tasks spread over the whole grid even for a small frontier.
//  Either way the edges of a round's vertices are expanded end to end
//  (td_expand), so the work of a task is balanced over the lanes whatever
//  the degree mix, and its dependent loads are shared.
//  * Vertices of degree > hub_deg are expanded chunk by chunk (2^chunk_log2
//    edges), 64 chunks per wavefront step, so a hub's edges spread over the
//    whole grid: from the list of the frontier's hubs, or from the table of
//    every hub chunk of the graph, keeping the chunks of frontier vertices.
// sink(uq, jq, okq) receives four (source, edge index) pairs per lane, with
// every lane of the wavefront active; okq marks the real ones.  The
// assignment of edges to wavefronts depends only on the frontier and its
// sources, so passes over the same frontier see the same edges in the same
// wavefronts.
template <class Sink>
__device__ __forceinline__ void td_scan(const Params &P, const unsigned long long *front, const FrontSrc &src, bool fold_vis,
                        long long gwave, long long nwaves, Sink &sink)
{
    const int lane = __lane_id();
    if (src.q) {
        const long long len = src.qlen;
        long long E = (len + nwaves - 1) / nwaves;
        E = E < 1 ? 1 : (E > 64 ? 64 : E);
        for (long long lo = gwave * E; lo < len; lo += nwaves * E) {
            int u = -1, dl = 0;
            long long sl = 0;
            if (lane < E && lo + lane < len) {
                u = src.q[lo + lane];
                if ((unsigned)u >= (unsigned)P.n) {   // would be a kernel bug: report it
                    atomicOr((unsigned *)&P.ctrl->status, 8u);
                    u = -1;
                } else {
                    // F_d joins the finished layers (other lanes may share the word)
                    if (fold_vis && src.q_fold) atomicOr(&P.vis[u >> 6], 1ull << (u & 63));
                    dl = P.deg[u];
                    sl = P.off[u];
                    if (dl > P.hub_deg) dl = 0;      // expanded chunk by chunk below
                }
            }
            td_expand(P, u, dl, sl, sink);
        }
    } else {
        const int G = P.wpg_td;
        for (long long base = gwave * G; base < P.W; base += nwaves * G) {
            const long long myw = base + lane;
            const unsigned long long fwl = (lane < G && myw < P.W) ? front[myw] : 0ull;
            if (fold_vis && fwl) P.vis[myw] |= fwl;  // F_d joins the finished layers (lane owns word)
            const int cnt = __popcll(fwl);
            const int cincl = wave_incl_scan32(cnt);
            const int cex = cincl - cnt;
            const int V = __builtin_amdgcn_readlane(cincl, 63);
            for (int vr = 0; vr < V; vr += 64) {
                // cross-lane reads run with every lane active (an inactive source
                // lane would read as 0); only lanes with vi < V use the result
                const int vi = vr + lane;
                const bool vok = vi < V;
                const int l = lane_search(cex, vok ? vi : 0);
                const unsigned long long fw = (unsigned long long)__shfl((long long)fwl, l);
                const int kth = vi - __shfl(cex, l);
                int u = -1, dl = 0;
                long long sl = 0;
                if (vok) {
                    u = (int)(((base + l) << 6) + select_bit(fw, kth));
                    if ((unsigned)u >= (unsigned)P.n) {   // would be a kernel bug: report it
                        atomicOr((unsigned *)&P.ctrl->status, 8u);
                        u = 0;
                    }
                    dl = P.deg[u];
                    sl = P.off[u];
                    if (dl > P.hub_deg) dl = 0;      // expanded chunk by chunk below
                }
                td_expand(P, u, dl, sl, sink);
            }
        }
    }
    // high-degree frontier vertices, 64 chunks per step, lane l of wavefront g
    // taking entry g + l * nwaves so that the adjacent chunks of one hub go to
    // different wavefronts
    const long long CH = 1ll << P.chunk_log2;
    const long long nh = src.nhubs;
    for (long long b0 = gwave; b0 < nh; b0 += nwaves * 64) {
        const long long idx = b0 + (long long)lane * nwaves;
        Item it{-1, 0};
        if (idx < nh) it = src.hubs[idx];
        // the table lists every vertex above the graph's cut-off; a vertex at
        // or below this run's cut-off was expanded with the flattened edges
        const bool hit =
            it.u >= 0 && (src.hubs_listed || (test_bit(front, it.u) && P.deg[it.u] > P.hub_deg));
        unsigned long long m = __ballot(hit);
        while (m) {
            const int k = __ffsll((long long)m) - 1;
            m &= m - 1;
            const int uh = __builtin_amdgcn_readlane(it.u, k);
            const int ch = __builtin_amdgcn_readlane(it.chunk, k);
            const long long s = P.off[uh] + ((long long)ch << P.chunk_log2);
            const long long e = min(s + CH, P.off[uh + 1]);
            for (long long r0 = s; r0 < e; r0 += 256) {
                int uq[4];
                long long jq[4];
                bool okq[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uq[q] = uh;
                    jq[q] = r0 + q * 64 + lane;
                    okq[q] = jq[q] < e;
                }
                sink(uq, jq, okq);
            }
        }
    }
}

// Top-down step (Algorithm 1) with canonical parents by atomic minimum.
__device__ __forceinline__ void top_down_step(const Params &P, int d, const unsigned long long *front,
                              unsigned long long *next, unsigned long long &nf,
                              unsigned long long &mf, unsigned long long &nh, const FrontSrc &src,
                              long long gwave, long long nwaves, HubStage *hs, WorkCount &wc)
{
    auto sink = [&](const int (&uq)[4], const long long (&jq)[4], const bool (&okq)[4]) {
        td_edges4(P, d, uq, jq, okq, front, next, nf, mf, nh, hs, wc);
    };
    td_scan(P, front, src, true, gwave, nwaves, sink);
}

// ---------------------------------------------------------------------------
// Bottom-up step.  A wavefront task covers G bitmap words; the words that
// still have unvisited vertices are taken two at a time, lane i handling
// vertex i of both, so the loads of two words overlap:
//   phase 1 (Algorithms 4-5): every unvisited lane tests the first positions
//            of its ascending row against the frontier bitmap -- the first
//            slab_k from the position-major slab (coalesced, issued together
//            with the degree load), the rest up to K from the column array,
//            four per round;
//   phase 2 (Algorithm 2 for the lanes left over): each unresolved row is
//            scanned by the whole wavefront, 64 entries per step, and the
//            first hit is taken with ballot + find-first-set.
// The first hit in ascending order is the canonical parent.
__device__ __forceinline__ void bu_finish_vertex(const Params &P, const unsigned long long *front,
                                                 const unsigned *lf, long long v, bool act, int dg, int KS,
                                                 int K, bool &found, int &par, WorkCount &wc)
{
    const int lane = __lane_id();
    // phase 1b: positions KS..K-1 from the column array
    long long s = 0;
    const bool need_s = act && !found && dg > KS;
    if (need_s) s = P.off[v];
    const long long e = s + dg;
    bool live = need_s && K > KS;
    for (int p0 = KS; p0 < K; p0 += 4) {
        if (!__ballot(live)) break;
        int c0 = -1, c1 = -1, c2 = -1, c3 = -1;
        if (live) {
            const long long b = s + p0;
            c0 = P.col[b];
            if (b + 1 < e && p0 + 1 < K) c1 = P.col[b + 1];
            if (b + 2 < e && p0 + 2 < K) c2 = P.col[b + 2];
            if (b + 3 < e && p0 + 3 < K) c3 = P.col[b + 3];
        }
        bool h0 = false, h1 = false, h2 = false, h3 = false;
        if (P.serial_probes) {
            h0 = c0 >= 0 && probe_front(front, lf, c0);
            h1 = !h0 && c1 >= 0 && probe_front(front, lf, c1);
            h2 = !h0 && !h1 && c2 >= 0 && probe_front(front, lf, c2);
            h3 = !h0 && !h1 && !h2 && c3 >= 0 && probe_front(front, lf, c3);
            if (P.count)
                wc.c[1] += (c0 >= 0) + (!h0 && c1 >= 0) + (!h0 && !h1 && c2 >= 0) + (!h0 && !h1 && !h2 && c3 >= 0);
        } else {
            if (P.count) wc.c[1] += (c0 >= 0) + (c1 >= 0) + (c2 >= 0) + (c3 >= 0);
            if (c0 >= 0) h0 = probe_front(front, lf, c0);
            if (c1 >= 0) h1 = probe_front(front, lf, c1);
            if (c2 >= 0) h2 = probe_front(front, lf, c2);
            if (c3 >= 0) h3 = probe_front(front, lf, c3);
        }
        if (live) {
            if (h0) { found = true; par = c0; }
            else if (h1) { found = true; par = c1; }
            else if (h2) { found = true; par = c2; }
            else if (h3) { found = true; par = c3; }
            if (found || s + p0 + 4 >= e) live = false;
        }
    }
    // phase 2: the rest of each unresolved row.  Rows with at most 32 entries
    // left go two to a step, one per half-wavefront; the others one at a time
    // over the whole wavefront.
    const int KP = max(K, KS);
    const bool cont = need_s && !found && dg > KP;
    unsigned long long rem = __ballot(cont);
    if (P.count && lane == 0) wc.c[2] += __popcll(rem);
    unsigned long long shrt = __ballot(cont && dg - KP <= 32);
    rem &= ~shrt;
    while (shrt) {
        const int ka = __ffsll((long long)shrt) - 1;
        shrt &= shrt - 1;
        int kb = -1;
        if (shrt) {
            kb = __ffsll((long long)shrt) - 1;
            shrt &= shrt - 1;
        }
        const long long sa = bcast64(s, ka) + KP, ea = bcast64(e, ka);
        long long sb = 0, eb = 0;
        if (kb >= 0) {
            sb = bcast64(s, kb) + KP;
            eb = bcast64(e, kb);
        }
        const bool hi = lane >= 32;
        const long long j = (hi ? sb : sa) + (lane & 31);
        const long long ej = hi ? eb : ea;
        int u = 0;
        bool hit = false;
        if (j < ej) {
            u = P.col[j];
            hit = probe_front(front, lf, u);
        }
        if (P.count) {
            wc.c[3] += lane == 0;
            wc.c[4] += j < ej;
        }
        const unsigned long long hb = __ballot(hit);
        const unsigned long long hlo = hb & 0xFFFFFFFFull, hhi = hb >> 32;
        const int hva = hlo ? __builtin_amdgcn_readlane(u, __ffsll((long long)hlo) - 1) : -1;
        const int hvb = hhi ? __builtin_amdgcn_readlane(u, 32 + __ffsll((long long)hhi) - 1) : -1;
        if (lane == ka && hva >= 0) {
            found = true;
            par = hva;
        }
        if (lane == kb && hvb >= 0) {
            found = true;
            par = hvb;
        }
    }
    while (rem) {
        const int k = __ffsll((long long)rem) - 1;
        rem &= rem - 1;
        const long long sk = bcast64(s, k) + KP;
        const long long ek = bcast64(e, k);
        int hitv = -1;
        for (long long b = sk; b < ek; b += 64) {
            const long long j = b + lane;
            int u = 0;
            bool hit = false;
            if (j < ek) {
                u = P.col[j];
                hit = probe_front(front, lf, u);
            }
            if (P.count) {
                wc.c[3] += lane == 0;
                wc.c[4] += j < ek;
            }
            const unsigned long long hb = __ballot(hit);
            if (hb) {
                hitv = __builtin_amdgcn_readlane(u, __ffsll((long long)hb) - 1);
                break;
            }
        }
        if (hitv >= 0 && lane == k) {
            found = true;
            par = hitv;
        }
    }
}

__device__ __forceinline__ void bottom_up_step(const Params &P, int d, const unsigned long long *front,
                               unsigned long long *next, unsigned long long &nf,
                               unsigned long long &mf, unsigned long long &nh, long long gwave,
                               long long nwaves, HubStage *hs, const unsigned *lf, WorkCount &wc)
{
    const int lane = __lane_id();
    const int K = P.probe_k;
    const int KS = min(P.slab_k, K);
    const int G = P.wpg;
    for (long long base = gwave * G; base < P.W; base += nwaves * G) {
        const long long myw = base + lane;
        const bool inr = lane < G && myw < P.W;
        unsigned long long vwl = ~0ull, fwl = 0ull;
        if (inr) {
            vwl = P.vis[myw];
            fwl = front[myw];
        }
        // fully seen words only need the frontier folded into vis
        if (inr && (fwl & ~vwl) && ((vwl | fwl) == ~0ull)) P.vis[myw] = vwl | fwl;
        unsigned long long todo = __ballot((vwl | fwl) != ~0ull);
        unsigned long long tfm = 0;   // lane l: vertices found in word base + l
        while (todo) {
            int wi[2];
            wi[0] = __ffsll((long long)todo) - 1;
            todo &= todo - 1;
            wi[1] = -1;
            if (todo) {
                wi[1] = __ffsll((long long)todo) - 1;
                todo &= todo - 1;
            }
            unsigned long long seen[2], vw[2];
            long long v[2];
            bool act[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                seen[j] = wi[j] >= 0 ? bcast_u64(vwl | fwl, wi[j]) : ~0ull;
                vw[j] = wi[j] >= 0 ? bcast_u64(vwl, wi[j]) : ~0ull;
                v[j] = ((base + (wi[j] >= 0 ? wi[j] : 0)) << 6) + lane;
                act[j] = !((seen[j] >> lane) & 1ull);
            }
            // phase 1a for both vertices: degree and slab loads together
            int dg[2], c[2][4];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                dg[j] = act[j] ? P.deg[v[j]] : 0;
#pragma unroll
                for (int p = 0; p < 4; ++p)
                    c[j][p] = (act[j] && p < KS) ? P.slab[(long long)p * P.n + v[j]] : -1;
            }
            bool found[2];
            int par[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                found[j] = false;
                par[j] = -1;
                if (P.count) wc.c[0] += act[j];
                if (P.serial_probes) {
                    // one frontier-bit probe at a time, none after the first hit
#pragma unroll
                    for (int p = 0; p < 4; ++p) {
                        if (P.count) wc.c[1] += !found[j] && c[j][p] >= 0;
                        if (!found[j] && c[j][p] >= 0 && probe_front(front, lf, c[j][p])) {
                            found[j] = true;
                            par[j] = c[j][p];
                        }
                    }
                    continue;
                }
                bool h[4];
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    h[p] = c[j][p] >= 0 && probe_front(front, lf, c[j][p]);
                    if (P.count) wc.c[1] += c[j][p] >= 0;
                }
#pragma unroll
                for (int p = 3; p >= 0; --p)
                    if (h[p]) {
                        found[j] = true;
                        par[j] = c[j][p];
                    }
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if (wi[j] < 0) continue;
                bu_finish_vertex(P, front, lf, v[j], act[j], dg[j], KS, K, found[j], par[j], wc);
                const unsigned long long fm = __ballot(found[j]);
                if (P.count) wc.c[5] += found[j];
                if (found[j]) {
                    P.level[v[j]] = d + 1;
                    P.parent[v[j]] = par[j];
                    nf += 1;
                    mf += (unsigned long long)dg[j];
                    nh += dg[j] > P.hub_deg;
                    if (P.h_write && dg[j] > P.hub_deg) hub_stage(hs, (int)v[j]);
                }
                if (lane == wi[j]) tfm = fm;
                // `next` was cleared one layer ahead: store only nonzero words
                if (lane == 0) {
                    const long long w = base + wi[j];
                    if (fm) next[w] = fm;
                    if ((seen[j] | fm) != vw[j]) P.vis[w] = seen[j] | fm;
                }
            }
        }
        // the task's part of F_{d+1} as a queue, in ascending order
        if (P.q_write) queue_append_words(P, d, base, tfm);
    }
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ void flush_counters(unsigned long long nf, unsigned long long mf, unsigned long long nh,
                               Slot *slot, unsigned long long *s_red, int nwaves_block)
{
    unsigned long long *sub = slot->c[blockIdx.x % kSub];
    const int lane = __lane_id();
    const int wib = threadIdx.x >> 6;
    nf = wave_sum_u64(nf);
    mf = wave_sum_u64(mf);
    nh = wave_sum_u64(nh);
    if (lane == 0) {
        s_red[3 * wib] = nf;
        s_red[3 * wib + 1] = mf;
        s_red[3 * wib + 2] = nh;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0, b = 0, c = 0;
        for (int i = 0; i < nwaves_block; ++i) {
            a += s_red[3 * i];
            b += s_red[3 * i + 1];
            c += s_red[3 * i + 2];
        }
        if (a) atomicAdd(&sub[0], a);
        if (b) atomicAdd(&sub[1], b);
        if (c) atomicAdd(&sub[2], c);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Binned top-down step for large top-down layers.  The frontier's edges
// (u, v) are bucketed by the destination tile v >> bin_log2, then one block
// per tile takes each vertex's smallest frontier neighbour with LDS atomics
// and writes the tile's levels, parents and next-frontier words together.
// The HBM traffic becomes streaming (rows, bucket writes and reads, tile-wide
// output runs) instead of one random gather and atomic per edge.  Passes:
//   count   (in the layer kernel): edges per tile, in an LDS histogram per
//           block, then one global add per nonzero tile;
//   scan    (one block): bucket offsets;
//   scatter: the same edge enumeration (same edges in the same wavefronts),
//           per-block ranges of each bucket reserved with one atomic per
//           (block, tile), pairs placed by LDS atomics;
//   reduce  : per tile, minima in LDS over unvisited targets, then output.

static __device__ __forceinline__ void bin_count_pass(const Params &P, const unsigned long long *front, unsigned *hist,
                                      const FrontSrc &src, long long gwave, long long nwaves)
{
    for (int b = threadIdx.x; b < P.nbins; b += blockDim.x) hist[b] = 0u;
    __syncthreads();
    auto sink = [&](const int (&uq)[4], const long long (&jq)[4], const bool (&okq)[4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (!okq[q]) continue;
            if ((unsigned long long)jq[q] >= (unsigned long long)P.nnz) {
                atomicOr((unsigned *)&P.ctrl->status, 4u);
                continue;
            }
            atomicAdd(&hist[P.col[jq[q]] >> P.bin_log2], 1u);
        }
    };
    td_scan(P, front, src, true, gwave, nwaves, sink);
    __syncthreads();
    for (int b = threadIdx.x; b < P.nbins; b += blockDim.x)
        if (hist[b]) atomicAdd(&P.bin_cnt[b], (int)hist[b]);
}

// Control data a block reads at the start of a layer.  It was written by
// earlier kernels (or, in the finisher, by this block before a barrier), so
// plain loads see it; thread 0 loads it once and the block shares it.
struct LayerView {
    int done;
    int pad;
    int *level;
    int *parent;
    LayerState S;
    long long n_f, m_f, n_h;
    long long q_len, hq_len;         // entries of F_d's queue and hub list
};

// kBuild: which lists the build of the layer kernel keeps and reads (BUILD_*):
// none (the plain bitmap path, which pays no registers for them), hub lists,
// or frontier queues and hub lists.  The host picks the build per launch
// (layer_build): with hub lists for layer 1 only, layer 1 runs in the
// hub-list build and the other layers in the plain one.
// kFilter: the build keeps the membership filters of small frontiers (only the
// wide build, used where the frontier bitmap does not fit in the L2).
template <int kBuild, bool kFilter>
__device__ __forceinline__ bool run_layer(const Params &Pin, int parity, long long gwave, long long nwaves,
                          long long gt, long long nt, bool leader, unsigned long long *s_red,
                          int nwaves_block, LayerView *view, bool same_kernel, int d_hint,
                          unsigned *hist, bool allow_binned, HubStage *hs)
{
    Ctrl *C = Pin.ctrl;
    if (threadIdx.x == 0) {
        if (kBuild != BUILD_PLAIN) hub_stage_reset(hs);
        view->done = C->done;
        view->level = C->level;
        view->parent = C->parent;
        view->S = C->st[parity];
        // kernel i of the launch sequence handles layer i, so its counter slot is
        // known without waiting for the state load; the finisher passes -1
        Slot &sl = C->slot[(d_hint >= 0 ? d_hint : view->S.d) % kSlots];
        long long a = 0, b = 0, c = 0;
        for (int k = 0; k < kSub; ++k) {
            // counters added by atomics earlier in this same kernel (finisher)
            // are read at the device-coherent level, past any stale L1 line
            a += (long long)(same_kernel ? ld_relaxed(&sl.c[k][0]) : sl.c[k][0]);
            b += (long long)(same_kernel ? ld_relaxed(&sl.c[k][1]) : sl.c[k][1]);
            c += (long long)(same_kernel ? ld_relaxed(&sl.c[k][2]) : sl.c[k][2]);
        }
        view->n_f = a;
        view->m_f = b;
        view->n_h = c;
        // list lengths only where the build reads lists
        view->q_len = kBuild != BUILD_QUEUES ? 0
                                             : (long long)(same_kernel ? ld_relaxed(&sl.c[0][kQueueTail])
                                                                       : sl.c[0][kQueueTail]);
        view->hq_len = kBuild == BUILD_PLAIN ? 0
                                             : (long long)(same_kernel ? ld_relaxed(&sl.c[0][kHubTail])
                                                                       : sl.c[0][kHubTail]);
    }
    __syncthreads();
    if (view->done) return false;
    // the outputs of this traversal were recorded by the init kernel
    Params P = Pin;
    P.level = view->level;
    P.parent = view->parent;
    if (kBuild != BUILD_QUEUES) P.td_queue = QM_OFF;
    if (kBuild == BUILD_PLAIN) P.hub_list = HL_OFF;
    if (kBuild != BUILD_COUNTS) P.count = 0;
    if (!kFilter) P.use_filter = 0;
    const LayerState S = view->S;
    const int d = S.d;
    if (d_hint >= 0 && d != d_hint) {
        // the launch sequence and the device state disagree: a host-side bug
        if (leader) atomicOr((unsigned *)&C->status, 16u);
        return false;
    }
    const long long n_f = view->n_f;
    const long long m_f = view->m_f;
    long long m_u = S.m_u, v_u = S.v_u;
    m_u -= m_f;
    v_u -= n_f;
    if (d > P.n) {
        // a BFS has at most n layers; stop with an error rather than loop
        if (leader) C->done = 2;
        return false;
    }
    if (n_f == 0) {
        if (leader) {
            C->nlayers = d;
            C->reached = S.reached;
            C->reached_deg = S.reached_deg;
            C->done = 1;
        }
        return false;
    }
    int cur = decide(P, S.dir_prev, n_f, m_f, m_u, v_u);
    // a layer that can run binned keeps top-down by its own alpha: the binned
    // step streams its edges through buckets instead of a random atomic per
    // edge, so it stays cheaper than a bottom-up scan for longer
    const bool can_bin = allow_binned && m_f >= P.bin_min_edges && m_f <= P.bin_cap;
    if (cur == DIR_BU && S.dir_prev == DIR_TD && P.rule == RULE_EDGES && can_bin && m_f * P.alpha_bin <= m_u)
        cur = DIR_TD;
    // a large top-down layer is bucketed by destination tile when the three
    // binned kernels follow this one (every block decides the same)
    const bool binned = can_bin && cur == DIR_TD;
    // where a top-down step finds F_d and its hubs
    FrontSrc src;
    src.q = nullptr;
    src.qlen = 0;
    src.q_fold = false;
    if (P.td_queue != QM_OFF && S.qform != QF_NONE) {
        if (view->q_len == n_f && n_f <= P.q_cap) {
            src.q = queue_of(P, d);
            src.qlen = n_f;
            src.q_fold = S.qform == QF_LIST;
        } else if (leader) {
            // every producer appends each vertex it discovers once: a queue
            // whose length differs from the frontier count is a kernel bug
            atomicOr((unsigned *)&C->status, 0x1000u);
        }
    }
    if (kBuild != BUILD_PLAIN && S.hlist && hub_list_usable(P, view->hq_len)) {
        src.hubs = hubs_of(P, d);
        src.nhubs = view->hq_len;
        src.hubs_listed = true;
    } else {
        src.hubs = P.hub;
        src.nhubs = view->n_h > 0 ? P.n_hub : 0;
        src.hubs_listed = false;
    }
    // this layer also writes F_{d+1} as a queue, and lists its hubs
    P.q_write = P.td_queue == QM_ALL || (P.td_queue == QM_TOPDOWN && cur == DIR_TD && !binned);
    P.h_write = P.hub_list == HL_ALL || (P.hub_list == HL_TD && cur == DIR_TD) ||
                (P.hub_list == HL_EARLY && cur == DIR_TD && d == 1 && !binned);
    // a small top-down layer fills its output's membership filter, which a
    // bottom-up layer with a small frontier uses (in the LDS of the tile
    // histogram, so not in the finisher, which has none)
    P.f_write = P.use_filter && cur == DIR_TD && !binned && m_f <= kFilterMaxEdges;
    const bool use_filter = kFilter && cur == DIR_BU && S.filt && n_f <= kFilterMaxFrontier && hist != nullptr;
    if (leader) {
        C->bin_layer = binned ? d : -1;
        C->bin_qlen = src.q ? (int)src.qlen : -1;
        C->bin_hlist = src.hubs_listed;
        if (d < P.trace_cap) {
            LayerRec r;
            r.dir = cur;
            r.pad = 0;
            r.n_f = n_f;
            r.m_f = m_f;
            r.m_u = m_u;
            r.v_u = v_u;
            // no device clock is read anywhere in these kernels: a kernel that
            // merely contains one (even on a branch not taken) was measured
            // about 10 us slower per launch on gfx950; per-layer times come
            // from HIP events around the launches instead
            P.trace[d] = r;
        }
        LayerState Nx = S;
        Nx.d = d + 1;
        Nx.dir_prev = cur;
        Nx.m_u = m_u;
        Nx.v_u = v_u;
        Nx.reached = S.reached + n_f;
        Nx.reached_deg = S.reached_deg + m_f;
        // the bottom-up step writes its found vertices into vis itself
        Nx.qform = !P.q_write ? QF_NONE : (cur == DIR_BU ? QF_LIST_VIS : QF_LIST);
        Nx.hlist = P.h_write;                // this layer lists the hubs it discovers
        Nx.filt = P.f_write;
        C->st[parity ^ 1] = Nx;
        C->parity = parity ^ 1;
        Slot *Z = &C->slot[(d + 2) % kSlots];
        for (int k = 0; k < kSub; ++k) {
            Z->c[k][0] = 0;
            Z->c[k][1] = 0;
            Z->c[k][2] = 0;
        }
        Z->c[0][kHubTail] = 0;
        Z->c[0][kQueueTail] = 0;
    }
    unsigned long long *front = P.bm + (long long)(d % 3) * P.W;
    unsigned long long *next = P.bm + (long long)((d + 1) % 3) * P.W;
    unsigned long long *spare = P.bm + (long long)((d + 2) % 3) * P.W;
    unsigned long long nf = 0, mf = 0, nh = 0;
    if (P.use_filter)
        for (long long w = gt; w < kFilterWords; w += nt) filt_of(P, d + 2)[w] = 0u;   // F_{d+2}'s filter
    if (use_filter) {
        const unsigned *gf = filt_of(P, d);
        for (int i = threadIdx.x; i < kFilterWords; i += nwaves_block * 64) hist[i] = gf[i];
        __syncthreads();
    }
    WorkCount wc;
#pragma unroll
    for (int k = 0; k < kCounts; ++k) wc.c[k] = 0;
    if (binned) bin_count_pass(P, front, hist, src, gwave, nwaves);
    else if (cur == DIR_TD) top_down_step(P, d, front, next, nf, mf, nh, src, gwave, nwaves, hs, wc);
    else bottom_up_step(P, d, front, next, nf, mf, nh, gwave, nwaves, hs, use_filter ? hist : nullptr, wc);
    if (P.count && d < P.trace_cap) {
#pragma unroll
        for (int k = 0; k < kCounts; ++k) {
            const unsigned long long t = wave_sum_u64(wc.c[k]);
            if (__lane_id() == 0 && t) atomicAdd(&P.pstat[(long long)d * kCounts + k], t);
        }
    }
    if (P.h_write) hub_flush(P, hs, d, nwaves_block);
    for (long long w = gt; w < P.W; w += nt) spare[w] = 0ull;   // `next` of layer d+1
    flush_counters(nf, mf, nh, &C->slot[(d + 1) % kSlots], s_red, nwaves_block);
    return true;
}

// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) bfs_init_kernel(Params P)
{
    const long long gt = (long long)blockIdx.x * kBlock + threadIdx.x;
    const long long nt = (long long)gridDim.x * kBlock;
    const int root = P.root;
    const long long rw = root >> 6;
    const unsigned long long rbit = 1ull << (root & 63);
    // 16-byte stores only when both outputs are 16-byte aligned
    const bool vec = ((((unsigned long long)P.level) | ((unsigned long long)P.parent)) & 15ull) == 0;
    const long long n4 = vec ? (P.n >> 2) : 0;
    int4 *l4 = (int4 *)P.level;
    int4 *p4 = (int4 *)P.parent;
    for (long long i = gt; i < n4; i += nt) {
        int4 a = make_int4(-1, -1, -1, -1), b = a;
        if (i == (root >> 2)) {
            const int c = root & 3;
            if (c == 0) { a.x = 0; b.x = root; }
            if (c == 1) { a.y = 0; b.y = root; }
            if (c == 2) { a.z = 0; b.z = root; }
            if (c == 3) { a.w = 0; b.w = root; }
        }
        l4[i] = a;
        p4[i] = b;
    }
    for (long long i = (n4 << 2) + gt; i < P.n; i += nt) {
        P.level[i] = i == root ? 0 : -1;
        P.parent[i] = i == root ? root : -1;
    }
    for (long long w = gt; w < P.W; w += nt) {
        const unsigned long long rb = (w == rw) ? rbit : 0ull;
        P.vis[w] = P.iso[w];                 // the root joins vis when layer 0 runs
        P.bm[w] = rb;                        // F_0 = {root}
        P.bm[P.W + w] = 0ull;                // next of layer 0
    }
    const long long deg_r = P.off[root + 1] - P.off[root];
    const bool root_hub = P.hub_list != HL_OFF && deg_r > P.hub_deg;
    long long root_chunks = root_hub ? (deg_r + (1ll << P.chunk_log2) - 1) >> P.chunk_log2 : 0;
    if (root_chunks > hub_list_limit(P)) root_chunks = -1;   // too long: layer 0 scans the table
    for (long long c = gt; c < root_chunks; c += nt) hubs_of(P, 0)[c] = Item{root, (int)c};   // F_0's hub list
    if (P.use_filter)
        for (long long w = gt; w < 3 * kFilterWords; w += nt) P.filt[w] = 0u;              // no filters yet
    if (P.count)
        for (long long i = gt; i < (long long)P.trace_cap * kCounts; i += nt) P.pstat[i] = 0ull;
    if (gt == 0) {
        Ctrl *C = P.ctrl;
        C->async_run = P.async_run;
        C->fail_injected = P.fail_injected;
        C->level = P.level;
        C->parent = P.parent;
        C->root = root;
        C->done = 0;
        C->nlayers = 0;
        C->parity = 0;
        C->reached = 0;
        C->reached_deg = 0;
        LayerState S;
        S.d = 0;
        S.dir_prev = DIR_TD;                 // Algorithm 3 starts top-down
        S.m_u = P.nnz;                       // layer 0 subtracts the root's own counts
        S.v_u = P.n;
        S.reached = 0;
        S.reached_deg = 0;
        S.qform = P.td_queue != QM_OFF ? QF_LIST : QF_NONE;
        S.hlist = P.hub_list != HL_OFF && root_chunks >= 0;
        S.filt = 0;
        S.pad1 = 0;
        S.pad[0] = 0;
        C->st[0] = S;
        C->st[1] = S;
        C->status = 0;
        if (P.td_queue != QM_OFF) queue_of(P, 0)[0] = root;   // F_0 as a queue
        for (int k = 0; k < kSlots; ++k)
            for (int j = 0; j < kSub; ++j)
                for (int e = 0; e < 8; ++e) C->slot[k].c[j][e] = 0ull;
        C->slot[0].c[0][0] = 1ull;
        C->slot[0].c[0][1] = (unsigned long long)deg_r;
        C->slot[0].c[0][2] = deg_r > P.hub_deg ? 1ull : 0ull;
        C->slot[0].c[0][kQueueTail] = P.td_queue != QM_OFF ? 1ull : 0ull;
        C->slot[0].c[0][kHubTail] =
            root_chunks < 0 ? (unsigned long long)hub_list_limit(P) + 1 : (unsigned long long)root_chunks;
    }
}

// One layer over the whole grid; the body of both builds of the layer kernel.
template <int kBuild, bool kFilter>
__device__ __forceinline__ void layer_grid(const Params &P, int layer, int allow_binned,
                                           unsigned long long *s_red, LayerView *view, unsigned *hist,
                                           HubStage *hs)
{
    const int parity = layer & 1;
    const long long gwave = (long long)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const long long nwaves = (long long)gridDim.x * kWavesPerBlock;
    const long long gt = (long long)blockIdx.x * kBlock + threadIdx.x;
    const long long nt = (long long)gridDim.x * kBlock;
    run_layer<kBuild, kFilter>(P, parity, gwave, nwaves, gt, nt, blockIdx.x == 0 && threadIdx.x == 0, s_red,
              kWavesPerBlock, view, false, layer, hist, allow_binned != 0 && P.nbins <= kMaxBins, hs);
}

template <int kBuild>
__global__ void __launch_bounds__(kBlock) bfs_layer_kernel(Params P, int layer, int allow_binned)
{
    __shared__ unsigned long long s_red[3 * kWavesPerBlock];
    __shared__ LayerView view;
    __shared__ unsigned hist[kMaxBins];
    __shared__ HubStage hs;
    layer_grid<kBuild, false>(P, layer, allow_binned, s_red, &view, hist, &hs);
}

// The same kernel built for kWideWavesPerSimd resident wavefronts per SIMD:
// fewer registers (a few values spill), more wavefronts in flight.  On graphs
// whose frontier bitmap no longer fits the L2, the layers are chains of
// dependent probes and row loads, and more chains in flight win; on smaller
// graphs the spills cost more than the extra wavefronts gain.
template <int kBuild, bool kFilter>
__global__ void __launch_bounds__(kBlock, kWideWavesPerSimd) bfs_layer_kernel_wide(Params P, int layer,
                                                                                  int allow_binned)
{
    __shared__ unsigned long long s_red[3 * kWavesPerBlock];
    __shared__ LayerView view;
    __shared__ unsigned hist[kMaxBins];
    __shared__ HubStage hs;
    layer_grid<kBuild, kFilter>(P, layer, allow_binned, s_red, &view, hist, &hs);
}

// One block runs whatever layers remain, with block barriers between them.
// One block of kFinisherBlock threads: half the size of the other one-block
// kernels, so that run_layer fits in its registers without spilling (a
// kernel with spills pays for private-memory setup at every launch, and the
// finisher runs after every traversal).
template <int kBuild>
__global__ void __launch_bounds__(kFinisherBlock) bfs_finish_kernel(Params P)
{
    __shared__ unsigned long long s_red[3 * (kFinisherBlock / 64)];
    __shared__ int s_parity;
    __shared__ LayerView view;
    __shared__ HubStage hs;
    const long long gwave = threadIdx.x >> 6;
    const long long nwaves = kFinisherBlock / 64;
    for (;;) {
        if (threadIdx.x == 0) s_parity = P.ctrl->parity;
        __syncthreads();
        const int parity = s_parity;
        if (!run_layer<kBuild, false>(P, parity, gwave, nwaves, threadIdx.x, kFinisherBlock, threadIdx.x == 0,
                                      s_red, kFinisherBlock / 64, &view, true, -1, nullptr, false, &hs))
            break;
        __syncthreads();
    }
    // the traversal is over: leave every counter slot at zero, so that the
    // next traversal on this workspace may add layer-1 counts in its first kernel
    __syncthreads();
    unsigned long long *c = &P.ctrl->slot[0].c[0][0];
    constexpr int kCounters = (int)(sizeof(Slot) / sizeof(unsigned long long)) * kSlots;
    for (int i = threadIdx.x; i < kCounters; i += kFinisherBlock) c[i] = 0ull;
    if (threadIdx.x == 0) record_failure(P.ctrl);
}

// Bucket offsets of a binned layer (one block): exclusive scan of the
// per-tile counts; the counts are cleared for the next binned layer.
__global__ void __launch_bounds__(kFinishBlock) bfs_bin_scan_kernel(Params P, int layer)
{
    __shared__ int s_part[kFinishBlock];
    Ctrl *C = P.ctrl;
    if (C->bin_layer != layer) return;
    const int per = (P.nbins + kFinishBlock - 1) / kFinishBlock;
    const int b0 = threadIdx.x * per;
    int sum = 0;
    for (int b = b0; b < b0 + per && b < P.nbins; ++b) sum += P.bin_cnt[b];
    s_part[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int i = 0; i < kFinishBlock; ++i) {
            const int t = s_part[i];
            s_part[i] = acc;
            acc += t;
        }
        P.bin_off[P.nbins] = acc;
        if ((long long)acc > P.bin_cap) {
            // cannot happen: the layer was binned only when m_f <= bin_cap
            atomicOr((unsigned *)&C->status, 64u);
            C->bin_layer = -2;
        }
    }
    __syncthreads();
    int acc = s_part[threadIdx.x];
    for (int b = b0; b < b0 + per && b < P.nbins; ++b) {
        const int c = P.bin_cnt[b];
        P.bin_off[b] = acc;
        P.bin_cur[b] = acc;
        P.bin_cnt[b] = 0;
        acc += c;
    }
}

__global__ void __launch_bounds__(kBlock) bfs_bin_scatter_kernel(Params P, int layer)
{
    __shared__ unsigned lbase[kMaxBins];
    __shared__ int s_go;
    __shared__ int s_qlen;
    __shared__ int s_hlist;
    __shared__ unsigned long long s_hubs, s_hq;
    Ctrl *C = P.ctrl;
    if (threadIdx.x == 0) {
        s_go = C->bin_layer == layer && P.nbins <= kMaxBins;
        s_qlen = C->bin_qlen;
        unsigned long long h = 0;
        const Slot &sl = C->slot[layer % kSlots];
        for (int k = 0; k < kSub; ++k) h += sl.c[k][2];
        s_hubs = h;
        s_hq = sl.c[0][kHubTail];
        s_hlist = C->bin_hlist;
    }
    __syncthreads();
    if (!s_go) return;
    const long long gwave = (long long)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const long long nwaves = (long long)gridDim.x * kWavesPerBlock;
    const unsigned long long *front = P.bm + (long long)(layer % 3) * P.W;
    // the frontier sources the layer kernel's count pass used
    FrontSrc src;
    src.q = s_qlen >= 0 ? queue_of(P, layer) : nullptr;
    src.qlen = s_qlen >= 0 ? s_qlen : 0;
    src.q_fold = false;
    const bool listed = s_hlist && hub_list_usable(P, (long long)s_hq);
    src.hubs = listed ? hubs_of(P, layer) : P.hub;
    src.nhubs = listed ? (long long)s_hq : (s_hubs > 0 ? P.n_hub : 0);
    src.hubs_listed = listed;
    // this block's edges per tile, then a range of each bucket for them
    for (int b = threadIdx.x; b < P.nbins; b += blockDim.x) lbase[b] = 0u;
    __syncthreads();
    auto count = [&](const int (&uq)[4], const long long (&jq)[4], const bool (&okq)[4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (okq[q] && (unsigned long long)jq[q] < (unsigned long long)P.nnz)
                atomicAdd(&lbase[P.col[jq[q]] >> P.bin_log2], 1u);
    };
    td_scan(P, front, src, false, gwave, nwaves, count);
    __syncthreads();
    for (int b = threadIdx.x; b < P.nbins; b += blockDim.x) {
        const unsigned c = lbase[b];
        lbase[b] = c ? (unsigned)atomicAdd(&P.bin_cur[b], (int)c) : 0u;
    }
    __syncthreads();
    const unsigned mask = (1u << P.bin_log2) - 1u;
    auto place = [&](const int (&uq)[4], const long long (&jq)[4], const bool (&okq)[4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (!okq[q] || (unsigned long long)jq[q] >= (unsigned long long)P.nnz) continue;
            const int v = P.col[jq[q]];
            const int b = v >> P.bin_log2;
            const unsigned pos = atomicAdd(&lbase[b], 1u);
            if ((int)pos < P.bin_off[b + 1])
                P.bin_pairs[pos] = ((unsigned long long)(unsigned)uq[q] << 32) | (unsigned)(v & mask);
            else
                atomicOr((unsigned *)&C->status, 64u);
        }
    };
    td_scan(P, front, src, false, gwave, nwaves, place);
}

// Two blocks of this size and their 64 KiB tiles fit one CU, so one tile's
// loads overlap another's LDS work.
constexpr int kReduceBlock = kReduceBlockThreads;

// One block per destination tile: the smallest frontier neighbour of every
// unvisited vertex of the tile by LDS atomic minimum over its bucket, then
// level d+1, parent, next-frontier word and counters, a wavefront per word.
__global__ void __launch_bounds__(kReduceBlock) bfs_bin_reduce_kernel(Params P, int layer)
{
    __shared__ unsigned par[1 << kBinLog2];
    __shared__ unsigned long long visw[(1 << kBinLog2) / 64];
    __shared__ unsigned long long s_red[3 * (kReduceBlock / 64)];
    __shared__ int s_go;
    __shared__ int *s_level;
    __shared__ int *s_parent;
    __shared__ HubStage hs;
    Ctrl *C = P.ctrl;
    if (threadIdx.x == 0) {
        s_go = C->bin_layer == layer && P.bin_log2 == kBinLog2;
        s_level = C->level;
        s_parent = C->parent;
        hub_stage_reset(&hs);
    }
    __syncthreads();
    if (!s_go) return;
    int *level = s_level;
    int *parent = s_parent;
    const int d = layer;
    const int lane = __lane_id();
    const int wib = threadIdx.x >> 6;
    constexpr int T = 1 << kBinLog2;
    constexpr int TW = T / 64;
    unsigned long long *next = P.bm + (long long)((d + 1) % 3) * P.W;
    unsigned long long nf = 0, mf = 0, nh = 0;
    // the layer is top-down: it lists its hubs in both modes that list them there
    const bool hubs_out = P.hub_list == HL_ALL || P.hub_list == HL_TD;
    for (int tile = blockIdx.x; tile < P.nbins; tile += gridDim.x) {
        const long long v0 = (long long)tile << kBinLog2;
        const long long w0 = v0 >> 6;
        for (int i = threadIdx.x; i < T; i += kReduceBlock) par[i] = 0xFFFFFFFFu;
        for (int i = threadIdx.x; i < TW; i += kReduceBlock) visw[i] = w0 + i < P.W ? P.vis[w0 + i] : ~0ull;
        __syncthreads();
        // four pairs per thread per step, loads first
        const int e = P.bin_off[tile + 1];
        for (int i0 = P.bin_off[tile] + threadIdx.x; i0 < e; i0 += 4 * kReduceBlock) {
            unsigned long long pr[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = i0 + q * kReduceBlock;
                pr[q] = i < e ? P.bin_pairs[i] : ~0ull;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (pr[q] == ~0ull) continue;
                const unsigned vl = (unsigned)pr[q] & (unsigned)(T - 1);
                if (!((visw[vl >> 6] >> (vl & 63)) & 1ull)) atomicMin(&par[vl], (unsigned)(pr[q] >> 32));
            }
        }
        __syncthreads();
        // four words per wavefront per step, their degree loads issued together
        constexpr int NWB = kReduceBlock / 64;
        for (int wq = wib; wq < TW; wq += 4 * NWB) {
            long long v[4];
            unsigned p[4];
            bool found[4];
            int dv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int w = wq + q * NWB;
                v[q] = v0 + ((long long)w << 6) + lane;
                p[q] = w < TW ? par[(w << 6) + lane] : 0xFFFFFFFFu;
                found[q] = p[q] != 0xFFFFFFFFu && v[q] < P.n;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) dv[q] = found[q] ? P.deg[v[q]] : 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int w = wq + q * NWB;
                const unsigned long long um = __ballot(found[q]);
                if (lane == 0 && um && w0 + w < P.W) next[w0 + w] = um;
                if (found[q]) {
                    level[v[q]] = d + 1;
                    parent[v[q]] = (int)p[q];
                    nf += 1;
                    mf += (unsigned long long)dv[q];
                    nh += dv[q] > P.hub_deg;
                }
                if (hubs_out && found[q] && dv[q] > P.hub_deg) hub_stage(&hs, (int)v[q]);
            }
            if (P.td_queue == QM_ALL) {
                int vq[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) vq[q] = (int)v[q];
                queue_append4(P, d, found, vq);
            }
        }
        __syncthreads();
    }
    if (hubs_out) hub_flush(P, &hs, d, kReduceBlock / 64);
    flush_counters(nf, mf, nh, &C->slot[(d + 1) % kSlots], s_red, kReduceBlock / 64);
}

// Layer 0 in one block, for a root of small degree: F_0 = {root}, so the
// top-down step is the expansion of the root's own row (each neighbour's
// parent is the root; duplicates are settled by the next-frontier bit), and a
// whole-grid launch would spend its time on launch and a bitmap scan.  The
// direction Algorithm 3 picks for layer 0 is recorded as usual; a bottom-up
// step from {root} would find exactly the same vertices and parents.
// Layer 0's bookkeeping (F_0 = {root}, its degree deg_r): Algorithm 3's
// decision for the root's row, the layer's trace entry, and the state that
// layer 1 starts from.  S is the state before layer 0.
__device__ void layer0_state(const Params &P, Ctrl *C, const LayerState &S, long long deg_r)
{
    const long long m_u = S.m_u - deg_r, v_u = S.v_u - 1;
    const int cur = decide(P, S.dir_prev, 1, deg_r, m_u, v_u);
    C->bin_layer = -1;
    if (P.trace_cap > 0) {
        LayerRec r;
        r.dir = cur;
        r.pad = 0;
        r.n_f = 1;
        r.m_f = deg_r;
        r.m_u = m_u;
        r.v_u = v_u;
        P.trace[0] = r;
    }
    LayerState Nx = S;
    Nx.d = 1;
    Nx.dir_prev = cur;
    Nx.m_u = m_u;
    Nx.v_u = v_u;
    Nx.reached = 1;
    Nx.reached_deg = deg_r;
    Nx.qform = P.td_queue != QM_OFF ? QF_LIST : QF_NONE;   // F_1 is appended to its queue
    Nx.hlist = P.hub_list != HL_OFF;                        // and its hubs to its hub list
    Nx.filt = 0;
    C->st[1] = Nx;
    C->parity = 1;
}

// Per-BFS initialisation fused with layer 0, for a root of degree at most
// kRootKernelDegree.  Block b owns bitmap words [b*per, (b+1)*per) and their
// vertices: it writes their initial outputs and bitmap words, then takes the
// root's neighbours that fall in its range (every block reads the root's
// row), so each output entry and bitmap word is written by one block only
// and no ordering between blocks is needed.  Layer 1's counters are added
// here; they start at zero because the previous traversal's finisher cleared
// them, and the host uses this kernel only when that holds.
__global__ void __launch_bounds__(kBlock) bfs_init_root_kernel(Params P, int per)
{
    __shared__ unsigned long long s_next[kFuseWords];
    __shared__ unsigned long long s_red[3 * kWavesPerBlock];
    __shared__ HubStage hs;
    Ctrl *C = P.ctrl;
    if (threadIdx.x == 0) hub_stage_reset(&hs);
    const int root = P.root;
    const long long rw = root >> 6;
    const unsigned long long rbit = 1ull << (root & 63);
    const long long s0 = P.off[root], e0 = P.off[root + 1];
    const long long deg_r = e0 - s0;
    const long long w0 = min((long long)blockIdx.x * per, P.W);
    const long long w1 = min(w0 + per, P.W);
    const long long v0 = w0 << 6, v1 = min(w1 << 6, P.n);
    if (P.use_filter && blockIdx.x == 0)
        for (int w = threadIdx.x; w < 3 * kFilterWords; w += kBlock) P.filt[w] = 0u;   // no filters yet
    if (P.count)
        for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < (long long)P.trace_cap * kCounts;
             i += (long long)gridDim.x * kBlock)
            P.pstat[i] = 0ull;
    for (long long w = w0 + threadIdx.x; w < w1; w += kBlock) {
        const unsigned long long rb = (w == rw) ? rbit : 0ull;
        s_next[w - w0] = 0ull;
        P.vis[w] = P.iso[w] | rb;            // F_0 = {root} is finished after layer 0
        P.bm[w] = rb;
        P.bm[2 * P.W + w] = 0ull;            // `next` of layer 1
    }
    if (v0 < v1) {
        // outputs of the range: 16-byte stores when both arrays are 16-byte
        // aligned (v0 is a multiple of 64, so the range keeps the alignment);
        // a block past the last word owns nothing and writes nothing
        const bool vec = ((((unsigned long long)P.level) | ((unsigned long long)P.parent)) & 15ull) == 0;
        const long long q1 = vec ? (v1 >> 2) : (v0 >> 2);
        int4 *l4 = (int4 *)P.level;
        int4 *p4 = (int4 *)P.parent;
        for (long long q = (v0 >> 2) + threadIdx.x; q < q1; q += kBlock) {
            int4 a = make_int4(-1, -1, -1, -1), b = a;
            if (q == (root >> 2)) {
                const int c = root & 3;
                if (c == 0) { a.x = 0; b.x = root; }
                if (c == 1) { a.y = 0; b.y = root; }
                if (c == 2) { a.z = 0; b.z = root; }
                if (c == 3) { a.w = 0; b.w = root; }
            }
            l4[q] = a;
            p4[q] = b;
        }
        for (long long v = (q1 << 2) + threadIdx.x; v < v1; v += kBlock) {
            P.level[v] = v == root ? 0 : -1;
            P.parent[v] = v == root ? root : -1;
        }
    }
    __syncthreads();   // the range's -1 entries precede its layer-1 entries
    unsigned long long nf = 0, mf = 0, nh = 0;
    const int lane = __lane_id();
    // whole wavefronts step through the row together (the appends to F_1's
    // queue and hub list are per wavefront)
    for (long long jb = s0 + (threadIdx.x - lane); jb < e0; jb += kBlock) {
        const long long j = jb + lane;
        bool disc = false;
        int v = -1, dv = 0;
        if (j < e0) {
            v = P.col[j];
            if (v != root && v >= v0 && v < v1) {
                const unsigned long long bit = 1ull << (v & 63);
                const unsigned long long old = atomicOr(&s_next[(v >> 6) - w0], bit);   // LDS: repeated entries count once
                if (!(old & bit)) {
                    disc = true;
                    P.level[v] = 1;
                    P.parent[v] = root;
                    dv = P.deg[v];
                    nf += 1;
                    mf += (unsigned long long)dv;
                    nh += dv > P.hub_deg;
                }
            }
        }
        if (P.td_queue != QM_OFF) queue_append1(P, 0, disc, v);
        if (P.hub_list != HL_OFF && disc && dv > P.hub_deg) hub_stage(&hs, v);
    }
    if (P.hub_list != HL_OFF) hub_flush(P, &hs, 0, kWavesPerBlock);
    __syncthreads();
    for (long long w = w0 + threadIdx.x; w < w1; w += kBlock) P.bm[P.W + w] = s_next[w - w0];   // F_1
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // layer 0's control state and decision (Algorithm 3 starts top-down)
        LayerState S;
        S.d = 0;
        S.dir_prev = DIR_TD;
        S.m_u = P.nnz;
        S.v_u = P.n;
        S.reached = 0;
        S.reached_deg = 0;
        S.qform = QF_NONE;
        S.hlist = 0;
        S.filt = 0;
        S.pad1 = 0;
        S.pad[0] = 0;
        C->level = P.level;
        C->parent = P.parent;
        C->root = root;
        C->done = 0;
        C->nlayers = 0;
        C->reached = 0;
        C->reached_deg = 0;
        C->status = 0;
        C->async_run = P.async_run;
        C->fail_injected = P.fail_injected;
        C->st[0] = S;
        layer0_state(P, C, S, deg_r);
    }
    flush_counters(nf, mf, nh, &C->slot[1], s_red, kWavesPerBlock);
}

__global__ void __launch_bounds__(kFinishBlock) bfs_root_kernel(Params P)
{
    __shared__ unsigned long long s_red[3 * (kFinishBlock / 64)];
    __shared__ HubStage hs;
    Ctrl *C = P.ctrl;
    if (threadIdx.x == 0) hub_stage_reset(&hs);
    __syncthreads();
    const int root = P.root;
    const long long s0 = P.off[root], e0 = P.off[root + 1];
    const long long deg_r = e0 - s0;
    if (threadIdx.x == 0) {
        layer0_state(P, C, C->st[0], deg_r);
        P.vis[root >> 6] |= 1ull << (root & 63);      // F_0 joins the finished layers
    }
    for (long long w = threadIdx.x; w < P.W; w += kFinishBlock) P.bm[2 * P.W + w] = 0ull;   // `next` of layer 1
    unsigned long long *next = P.bm + P.W;
    unsigned long long nf = 0, mf = 0, nh = 0;
    const int lane = __lane_id();
    for (long long jb = s0 + (threadIdx.x - lane); jb < e0; jb += kFinishBlock) {
        const long long j = jb + lane;
        bool disc = false;
        int v = -1, dv = 0;
        if (j < e0) {
            v = P.col[j];
            if (v != root && (unsigned)v < (unsigned)P.n) {
                const unsigned long long bit = 1ull << (v & 63);
                const unsigned long long old = atomicOr(&next[v >> 6], bit);
                if (!(old & bit)) {
                    disc = true;
                    P.level[v] = 1;
                    P.parent[v] = root;
                    dv = P.deg[v];
                    nf += 1;
                    mf += (unsigned long long)dv;
                    nh += dv > P.hub_deg;
                }
            }
        }
        if (P.td_queue != QM_OFF) queue_append1(P, 0, disc, v);
        if (P.hub_list != HL_OFF && disc && dv > P.hub_deg) hub_stage(&hs, v);
    }
    if (P.hub_list != HL_OFF) hub_flush(P, &hs, 0, kFinishBlock / 64);
    flush_counters(nf, mf, nh, &C->slot[1], s_red, kFinishBlock / 64);
}

// Isolated-vertex template of the visited bitmap: degree 0 or beyond n.
__global__ void iso_template_kernel(const long long *off, long long n, long long W,
                                    unsigned long long *iso)
{
    const long long w = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= W) return;
    unsigned long long m = 0;
    for (int b = 0; b < 64; ++b) {
        const long long v = (w << 6) + b;
        if (v >= n || off[v + 1] == off[v]) m |= 1ull << b;
    }
    iso[w] = m;
}

hipError_t launch_init(const Params &p, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(bfs_init_kernel, dim3(grid), dim3(kBlock), 0, s, p);
    return hipGetLastError();
}

int layer_build(const Params &p, int layer)
{
    if (p.count) return BUILD_COUNTS;
    if (p.td_queue != QM_OFF) return BUILD_QUEUES;
    if (p.hub_list == HL_ALL || p.hub_list == HL_TD) return BUILD_HUBS;
    if (p.hub_list == HL_LAYER0 && layer == 1) return BUILD_HUBS;
    if (p.hub_list == HL_EARLY && (layer == 1 || layer == 2)) return BUILD_HUBS;
    return BUILD_PLAIN;
}

int finish_build(const Params &p)
{
    if (p.count) return BUILD_COUNTS;
    if (p.td_queue != QM_OFF) return BUILD_QUEUES;
    if (p.hub_list == HL_ALL || p.hub_list == HL_TD) return BUILD_HUBS;
    return BUILD_PLAIN;
}

bool layer_filter(const Params &p, int layer)
{
    // the filter of F_2 is written by layer 1 (a small top-down layer from the
    // root's neighbours) and read by layer 2; the other layers run without
    // its code and registers
    return p.wide && p.use_filter && (layer == 1 || layer == 2);
}

template <int B>
static void launch_layer_build(const Params &p, int layer, int allow_binned, int grid, hipStream_t s)
{
    if (p.wide && layer_filter(p, layer))
        hipLaunchKernelGGL((bfs_layer_kernel_wide<B, true>), dim3(grid), dim3(kBlock), 0, s, p, layer, allow_binned);
    else if (p.wide)
        hipLaunchKernelGGL((bfs_layer_kernel_wide<B, false>), dim3(grid), dim3(kBlock), 0, s, p, layer, allow_binned);
    else
        hipLaunchKernelGGL(bfs_layer_kernel<B>, dim3(grid), dim3(kBlock), 0, s, p, layer, allow_binned);
}

hipError_t launch_layer(const Params &p, int layer, int allow_binned, int grid, hipStream_t s)
{
    switch (layer_build(p, layer)) {
    case BUILD_COUNTS: launch_layer_build<BUILD_COUNTS>(p, layer, allow_binned, grid, s); break;
    case BUILD_QUEUES: launch_layer_build<BUILD_QUEUES>(p, layer, allow_binned, grid, s); break;
    case BUILD_HUBS: launch_layer_build<BUILD_HUBS>(p, layer, allow_binned, grid, s); break;
    default: launch_layer_build<BUILD_PLAIN>(p, layer, allow_binned, grid, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_bin_scan(const Params &p, int layer, hipStream_t s)
{
    hipLaunchKernelGGL(bfs_bin_scan_kernel, dim3(1), dim3(kFinishBlock), 0, s, p, layer);
    return hipGetLastError();
}

hipError_t launch_bin_scatter(const Params &p, int layer, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(bfs_bin_scatter_kernel, dim3(grid), dim3(kBlock), 0, s, p, layer);
    return hipGetLastError();
}

hipError_t launch_bin_reduce(const Params &p, int layer, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(bfs_bin_reduce_kernel, dim3(grid), dim3(kReduceBlock), 0, s, p, layer);
    return hipGetLastError();
}

hipError_t launch_init_root(const Params &p, int grid, int per, hipStream_t s)
{
    hipLaunchKernelGGL(bfs_init_root_kernel, dim3(grid), dim3(kBlock), 0, s, p, per);
    return hipGetLastError();
}

hipError_t launch_root(const Params &p, hipStream_t s)
{
    hipLaunchKernelGGL(bfs_root_kernel, dim3(1), dim3(kFinishBlock), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_finish(const Params &p, hipStream_t s)
{
    switch (finish_build(p)) {
    case BUILD_COUNTS: hipLaunchKernelGGL(bfs_finish_kernel<BUILD_COUNTS>, dim3(1), dim3(kFinisherBlock), 0, s, p); break;
    case BUILD_QUEUES: hipLaunchKernelGGL(bfs_finish_kernel<BUILD_QUEUES>, dim3(1), dim3(kFinisherBlock), 0, s, p); break;
    case BUILD_HUBS: hipLaunchKernelGGL(bfs_finish_kernel<BUILD_HUBS>, dim3(1), dim3(kFinisherBlock), 0, s, p); break;
    default: hipLaunchKernelGGL(bfs_finish_kernel<BUILD_PLAIN>, dim3(1), dim3(kFinisherBlock), 0, s, p); break;
    }
    return hipGetLastError();
}

hipError_t launch_iso_template(const long long *off, long long n, long long W,
                               unsigned long long *iso, hipStream_t s)
{
    const int tb = 256;
    const long long blocks = (W + tb - 1) / tb;
    hipLaunchKernelGGL(iso_template_kernel, dim3((unsigned)blocks), dim3(tb), 0, s, off, n, W, iso);
    return hipGetLastError();
}

void *kernel_ptr_init() { return (void *)bfs_init_kernel; }
template <int B>
static void *layer_ptr(bool wide, bool filter)
{
    if (!wide) return (void *)bfs_layer_kernel<B>;
    return filter ? (void *)bfs_layer_kernel_wide<B, true> : (void *)bfs_layer_kernel_wide<B, false>;
}

void *kernel_ptr_layer(bool wide, int build, bool filter)
{
    switch (build) {
    case BUILD_COUNTS: return layer_ptr<BUILD_COUNTS>(wide, filter);
    case BUILD_QUEUES: return layer_ptr<BUILD_QUEUES>(wide, filter);
    case BUILD_HUBS: return layer_ptr<BUILD_HUBS>(wide, filter);
    default: return layer_ptr<BUILD_PLAIN>(wide, filter);
    }
}
void *kernel_ptr_init_root() { return (void *)bfs_init_root_kernel; }
void *kernel_ptr_bin_scan() { return (void *)bfs_bin_scan_kernel; }
void *kernel_ptr_bin_scatter() { return (void *)bfs_bin_scatter_kernel; }
void *kernel_ptr_bin_reduce() { return (void *)bfs_bin_reduce_kernel; }

void *kernel_ptr_finish(int build)
{
    switch (build) {
    case BUILD_COUNTS: return (void *)bfs_finish_kernel<BUILD_COUNTS>;
    case BUILD_QUEUES: return (void *)bfs_finish_kernel<BUILD_QUEUES>;
    case BUILD_HUBS: return (void *)bfs_finish_kernel<BUILD_HUBS>;
    default: return (void *)bfs_finish_kernel<BUILD_PLAIN>;
    }
}

int layer_blocks_per_cu(bool wide)
{
    int occ = 0;
    const hipError_t e =
        wide ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, bfs_layer_kernel_wide<BUILD_PLAIN, false>, kBlock, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, bfs_layer_kernel<BUILD_PLAIN>, kBlock, 0);
    return e == hipSuccess ? occ : -1;
}

}  // namespace hybfs
