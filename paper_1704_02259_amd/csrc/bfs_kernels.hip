// gfx950 kernels of the hybrid BFS.  A traversal is one init kernel followed
// by one kernel per layer (Algorithm 3's loop body): every block of the layer
// kernel reads the counters of the current frontier, takes the same
// direction decision, and runs either the top-down expansion (Algorithm 1) or
// the bottom-up step (Algorithm 2 with the multiple-parents probes of
// Algorithms 4-5).  Kernel boundaries order the layers; there is no grid-wide
// barrier and no co-residency requirement.  A single-block finisher runs any
// layers left after the enqueued layer kernels (very deep graphs).
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

namespace hybfs {

#define AGENT __HIP_MEMORY_SCOPE_AGENT

__device__ __forceinline__ unsigned long long ld_relaxed(unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, AGENT);
}

__device__ __forceinline__ long long bcast64(long long x, int lane)
{
    int lo = __builtin_amdgcn_readlane((int)(x & 0xFFFFFFFFll), lane);
    int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
    return ((long long)hi << 32) | (unsigned int)lo;
}

__device__ __forceinline__ unsigned long long bcast_u64(unsigned long long x, int lane)
{
    return (unsigned long long)bcast64((long long)x, lane);
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

__device__ __forceinline__ bool test_bit(const unsigned long long *bm, int v)
{
    return (bm[v >> 6] >> (v & 63)) & 1ull;
}

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
// One frontier edge u -> v of a top-down layer.  v is a candidate when it is
// in no layer <= d (neither in vis nor in the frontier).  A plain read of
// parent[v] skips the atomic when a smaller frontier neighbour already won;
// the edge that replaces the initial -1 discovers v.
__device__ __forceinline__ void td_edge(const Params &P, int d, int u, int v,
                                        const unsigned long long *front, unsigned long long *next,
                                        unsigned long long &nf, unsigned long long &mf)
{
    const int w = v >> 6;
    const unsigned long long bit = 1ull << (v & 63);
    if ((P.vis[w] | front[w]) & bit) return;
    const unsigned p = (unsigned)P.parent[v];
    if ((unsigned)u >= p) return;
    const unsigned old = atomicMin((unsigned int *)&P.parent[v], (unsigned int)u);
    if (old == 0xFFFFFFFFu) {
        P.level[v] = d + 1;
        atomicOr(&next[w], bit);
        nf += 1;
        mf += (unsigned long long)(P.off[v + 1] - P.off[v]);
    }
}

// Top-down step: the frontier bitmap is scanned 64 words per wavefront
// iteration; each nonzero word's vertices are expanded by degree class
// (one lane per vertex up to small_deg, the whole wavefront per vertex up to
// hub_deg).  Vertices above hub_deg are expanded through the static hub-chunk
// table, so their edges are spread over the whole grid.
__device__ void top_down_step(const Params &P, int d, const unsigned long long *front,
                              unsigned long long *next, unsigned long long &nf,
                              unsigned long long &mf, long long gwave, long long nwaves)
{
    const int lane = __lane_id();
    const int G = P.wpg;
    for (long long base = gwave * G; base < P.W; base += nwaves * G) {
        const long long myw = base + lane;
        const unsigned long long fwl = (lane < G && myw < P.W) ? front[myw] : 0ull;
        unsigned long long nz = __ballot(fwl != 0ull);
        while (nz) {
            const int i = __ffsll((long long)nz) - 1;
            nz &= nz - 1;
            const long long w = base + i;
            const unsigned long long fw = bcast_u64(fwl, i);
            if (lane == 0) P.vis[w] |= fw;       // F_d joins the finished layers
            const bool mine = (fw >> lane) & 1ull;
            const int u = (int)((w << 6) + lane);
            long long s = 0, e = 0;
            if (mine) {
                s = P.off[u];
                e = P.off[u + 1];
            }
            const long long deg = e - s;
            // one lane per low-degree vertex
            if (mine && deg <= P.small_deg) {
                for (long long j = s; j < e; ++j) td_edge(P, d, u, P.col[j], front, next, nf, mf);
            }
            // the whole wavefront per medium-degree vertex
            unsigned long long med = __ballot(mine && deg > P.small_deg && deg <= P.hub_deg);
            while (med) {
                const int k = __ffsll((long long)med) - 1;
                med &= med - 1;
                const int uk = __builtin_amdgcn_readlane(u, k);
                const long long sk = bcast64(s, k), ek = bcast64(e, k);
                for (long long j = sk + lane; j < ek; j += 64)
                    td_edge(P, d, uk, P.col[j], front, next, nf, mf);
            }
        }
    }
    // high-degree frontier vertices: chunks of 2^hub_log2 edges over the grid
    for (long long c = gwave; c < P.n_hub; c += nwaves) {
        const Item it = P.hub[c];
        if (!test_bit(front, it.u)) continue;
        const long long s = P.off[it.u] + ((long long)it.chunk << P.hub_log2);
        const long long e = min(s + (1ll << P.hub_log2), P.off[it.u + 1]);
        for (long long j = s + lane; j < e; j += 64) td_edge(P, d, it.u, P.col[j], front, next, nf, mf);
    }
}

// ---------------------------------------------------------------------------
// Bottom-up step.  A wavefront loads 64 words of vis and of the frontier,
// then handles each word that still has unvisited vertices, one lane per
// vertex:
//   phase 1 (Algorithms 4-5): every unvisited lane tests positions 0..K-1 of
//            its own ascending row against the frontier bitmap, four
//            positions per round;
//   phase 2 (Algorithm 2 for the lanes left over): each unresolved row is
//            scanned by the whole wavefront, 64 entries per step, and the
//            first hit is taken with ballot + find-first-set.
// The first hit in ascending order is the canonical parent.
__device__ void bottom_up_step(const Params &P, int d, const unsigned long long *front,
                               unsigned long long *next, unsigned long long &nf,
                               unsigned long long &mf, long long gwave, long long nwaves)
{
    const int lane = __lane_id();
    const int K = P.probe_k;
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
        while (todo) {
            const int i = __ffsll((long long)todo) - 1;
            todo &= todo - 1;
            const long long w = base + i;
            const unsigned long long seen = bcast_u64(vwl | fwl, i);
            const unsigned long long vw = bcast_u64(vwl, i);
            const long long v = (w << 6) + lane;
            const bool act = !((seen >> lane) & 1ull);
            long long s = 0, e = 0;
            if (act) {
                s = P.off[v];
                e = P.off[v + 1];
            }
            bool found = false;
            int par = -1;
            bool live = act && s < e;
            for (int p0 = 0; p0 < K; p0 += 4) {
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
                if (c0 >= 0) h0 = test_bit(front, c0);
                if (c1 >= 0) h1 = test_bit(front, c1);
                if (c2 >= 0) h2 = test_bit(front, c2);
                if (c3 >= 0) h3 = test_bit(front, c3);
                if (live) {
                    if (h0) { found = true; par = c0; }
                    else if (h1) { found = true; par = c1; }
                    else if (h2) { found = true; par = c2; }
                    else if (h3) { found = true; par = c3; }
                    if (found || s + p0 + 4 >= e) live = false;
                }
            }
            unsigned long long rem = __ballot(act && !found && s + K < e);
            while (rem) {
                const int k = __ffsll((long long)rem) - 1;
                rem &= rem - 1;
                const long long sk = bcast64(s, k) + K;
                const long long ek = bcast64(e, k);
                int hitv = -1;
                for (long long b = sk; b < ek; b += 64) {
                    const long long j = b + lane;
                    int u = 0;
                    bool hit = false;
                    if (j < ek) {
                        u = P.col[j];
                        hit = test_bit(front, u);
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
            const unsigned long long fm = __ballot(found);
            if (found) {
                P.level[v] = d + 1;
                P.parent[v] = par;
                nf += 1;
                mf += (unsigned long long)(e - s);
            }
            // `next` was cleared one layer ahead: store only nonzero words
            if (lane == 0) {
                if (fm) next[w] = fm;
                if ((seen | fm) != vw) P.vis[w] = seen | fm;
            }
        }
    }
}

// ---------------------------------------------------------------------------
__device__ void flush_counters(unsigned long long nf, unsigned long long mf, Slot *slot,
                               unsigned long long *s_red, int nwaves_block)
{
    const int lane = __lane_id();
    const int wib = threadIdx.x >> 6;
    nf = wave_sum_u64(nf);
    mf = wave_sum_u64(mf);
    if (lane == 0) {
        s_red[2 * wib] = nf;
        s_red[2 * wib + 1] = mf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0, b = 0;
        for (int i = 0; i < nwaves_block; ++i) {
            a += s_red[2 * i];
            b += s_red[2 * i + 1];
        }
        if (a) atomicAdd(&slot->n_f, a);
        if (b) atomicAdd(&slot->m_f, b);
    }
    __syncthreads();
}

// One layer (the body of Algorithm 3's loop).  Returns false once the BFS is
// complete.  `leader` is the one thread that writes shared control state.
__device__ bool run_layer(const Params &Pin, int parity, long long gwave, long long nwaves,
                          long long gt, long long nt, bool leader, unsigned long long *s_red,
                          int nwaves_block)
{
    Ctrl *C = Pin.ctrl;
    if (__hip_atomic_load(&C->done, __ATOMIC_RELAXED, AGENT)) return false;
    // the outputs of this traversal were recorded by the init kernel
    Params P = Pin;
    P.level = C->level;
    P.parent = C->parent;
    const LayerState S = C->st[parity];
    const int d = S.d;
    const long long n_f = (long long)ld_relaxed(&C->slot[d % kSlots].n_f);
    const long long m_f = (long long)ld_relaxed(&C->slot[d % kSlots].m_f);
    long long m_u = S.m_u, v_u = S.v_u;
    m_u -= m_f;
    v_u -= n_f;
    if (d > P.n) {
        // a BFS has at most n layers; stop with an error rather than loop
        if (leader) __hip_atomic_store(&C->done, 2, __ATOMIC_RELAXED, AGENT);
        return false;
    }
    if (n_f == 0) {
        if (leader) {
            C->nlayers = d;
            C->reached = S.reached;
            C->reached_deg = S.reached_deg;
            C->t_end = (unsigned long long)wall_clock64();
            __hip_atomic_store(&C->done, 1, __ATOMIC_RELAXED, AGENT);
        }
        return false;
    }
    const int cur = decide(P, S.dir_prev, n_f, m_f, m_u, v_u);
    if (leader) {
        if (d < P.trace_cap) {
            LayerRec r;
            r.dir = cur;
            r.pad = 0;
            r.n_f = n_f;
            r.m_f = m_f;
            r.m_u = m_u;
            r.v_u = v_u;
            r.t = (unsigned long long)wall_clock64();
            P.trace[d] = r;
        }
        LayerState Nx = S;
        Nx.d = d + 1;
        Nx.dir_prev = cur;
        Nx.m_u = m_u;
        Nx.v_u = v_u;
        Nx.reached = S.reached + n_f;
        Nx.reached_deg = S.reached_deg + m_f;
        C->st[parity ^ 1] = Nx;
        C->parity = parity ^ 1;
        Slot *Z = &C->slot[(d + 2) % kSlots];
        Z->n_f = 0;
        Z->m_f = 0;
    }
    unsigned long long *front = P.bm + (long long)(d % 3) * P.W;
    unsigned long long *next = P.bm + (long long)((d + 1) % 3) * P.W;
    unsigned long long *spare = P.bm + (long long)((d + 2) % 3) * P.W;
    unsigned long long nf = 0, mf = 0;
    if (cur == DIR_TD) top_down_step(P, d, front, next, nf, mf, gwave, nwaves);
    else bottom_up_step(P, d, front, next, nf, mf, gwave, nwaves);
    for (long long w = gt; w < P.W; w += nt) spare[w] = 0ull;   // `next` of layer d+1
    flush_counters(nf, mf, &C->slot[(d + 1) % kSlots], s_red, nwaves_block);
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
    if (gt == 0) {
        Ctrl *C = P.ctrl;
        const long long deg_r = P.off[root + 1] - P.off[root];
        C->level = P.level;
        C->parent = P.parent;
        C->root = root;
        C->done = 0;
        C->nlayers = 0;
        C->parity = 0;
        C->reached = 0;
        C->reached_deg = 0;
        C->t_end = 0;
        LayerState S;
        S.d = 0;
        S.dir_prev = DIR_TD;                 // Algorithm 3 starts top-down
        S.m_u = P.nnz;                       // layer 0 subtracts the root's own counts
        S.v_u = P.n;
        S.reached = 0;
        S.reached_deg = 0;
        S.pad[0] = S.pad[1] = S.pad[2] = 0;
        C->st[0] = S;
        C->st[1] = S;
        for (int k = 0; k < kSlots; ++k) {
            C->slot[k].n_f = k == 0 ? 1ull : 0ull;
            C->slot[k].m_f = k == 0 ? (unsigned long long)deg_r : 0ull;
        }
    }
}

__global__ void __launch_bounds__(kBlock) bfs_layer_kernel(Params P, int parity)
{
    __shared__ unsigned long long s_red[2 * kWavesPerBlock];
    const long long gwave = (long long)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const long long nwaves = (long long)gridDim.x * kWavesPerBlock;
    const long long gt = (long long)blockIdx.x * kBlock + threadIdx.x;
    const long long nt = (long long)gridDim.x * kBlock;
    run_layer(P, parity, gwave, nwaves, gt, nt, blockIdx.x == 0 && threadIdx.x == 0, s_red,
              kWavesPerBlock);
}

// One block runs whatever layers remain, with block barriers between them.
__global__ void __launch_bounds__(kFinishBlock) bfs_finish_kernel(Params P)
{
    __shared__ unsigned long long s_red[2 * (kFinishBlock / 64)];
    __shared__ int s_parity;
    const long long gwave = threadIdx.x >> 6;
    const long long nwaves = kFinishBlock / 64;
    for (;;) {
        if (threadIdx.x == 0) s_parity = __hip_atomic_load(&P.ctrl->parity, __ATOMIC_RELAXED, AGENT);
        __syncthreads();
        const int parity = s_parity;
        if (!run_layer(P, parity, gwave, nwaves, threadIdx.x, kFinishBlock, threadIdx.x == 0, s_red,
                       kFinishBlock / 64))
            break;
        __syncthreads();
    }
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

hipError_t launch_layer(const Params &p, int parity, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(bfs_layer_kernel, dim3(grid), dim3(kBlock), 0, s, p, parity);
    return hipGetLastError();
}

hipError_t launch_finish(const Params &p, hipStream_t s)
{
    hipLaunchKernelGGL(bfs_finish_kernel, dim3(1), dim3(kFinishBlock), 0, s, p);
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
void *kernel_ptr_layer() { return (void *)bfs_layer_kernel; }
void *kernel_ptr_finish() { return (void *)bfs_finish_kernel; }

int layer_blocks_per_cu()
{
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, bfs_layer_kernel, kBlock, 0) != hipSuccess)
        return -1;
    return occ;
}

}  // namespace hybfs
