// gfx950 kernels of the batched multi-source BFS: up to 64 roots traverse one
// graph together, lane b of a per-vertex uint64 mask standing for root b, so
// a row read once serves every root (adjacency reads are shared).  Outputs
// equal 64 single-root runs: level[b][v] and the canonical (smallest-id)
// parent of v in root b's tree.
//
// Per layer d two kernels run:
//   push (top-down layers only, Algorithm 1 on masks): every vertex u in any
//        lane's frontier sends fm_front[u] & ~vis[v] to each neighbour v --
//        one pass over u's row for all 64 roots; per lane, the parent of v is
//        the smallest such u (an unsigned atomic minimum);
//   pull (every layer): after a push, the vertices the push marked are folded
//        into vis and counted; in a bottom-up layer (Algorithm 2 on masks)
//        each vertex with lanes still unvisited scans its ascending row and
//        the first u whose frontier mask holds lane b is lane b's parent.
// Every block of both kernels reads the layer's counters and takes the same
// direction decision (Algorithm 3 on counts over the union of the lanes'
// frontiers), as in the single-root path.  The frontier masks of the first
// kBatchHist layers are kept, and after the finisher a level pass stores
// those layers' levels (and -1 where a root never arrived) in one coalesced
// sweep; deeper levels are stored by the layers that reach them.
#include "bfs_device.h"
#include "bfs_wave.h"

namespace hybfs {

static __device__ __forceinline__ unsigned long long wave_or_u64(unsigned long long x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o);
    return x;
}

// OR of x over the lanes below this one (all lanes active).
static __device__ __forceinline__ unsigned long long wave_excl_or(unsigned long long x)
{
    const int lane = __lane_id();
    unsigned long long incl = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long y = __shfl_up(incl, (unsigned)o);
        if (lane >= o) incl |= y;
    }
    const unsigned long long ex = __shfl_up(incl, 1u);
    return lane == 0 ? 0ull : ex;
}

// Direction from counts summed over the lanes; the table rule needs per-lane
// vertex counts and is taken as the edge rule here.
static __device__ __forceinline__ int bdecide(const BParams &P, int cur, long long u_nf, long long u_mf,
                                              long long m_u)
{
    if (P.rule == RULE_TOPDOWN) return DIR_TD;
    if (P.rule == RULE_BOTTOMUP) return DIR_BU;
    if (cur == DIR_TD && u_mf * P.alpha > m_u) return DIR_BU;
    if (cur == DIR_BU && u_nf * P.beta < P.n) return DIR_TD;
    return cur;
}

// Where F_d's lane masks live: the first P.hist layers keep their own slots
// until the level pass has read them; later layers rotate through the three
// slots after those.
static __device__ __forceinline__ unsigned long long *fmask(const BParams &P, int d)
{
    const long long slot = d < P.hist ? d : P.hist + (d - P.hist) % 3;
    return P.fm + slot * P.n;
}

// Whether level d is stored by the layer that reaches it (d >= P.hist); the
// levels below P.hist are stored by the level pass from the kept masks.
static __device__ __forceinline__ bool layer_stores_level(const BParams &P, int d) { return d >= P.hist; }

// Lane b of `bits`: v's parent in root b's tree is u.  (The levels of a
// bottom-up layer are stored afterwards, per lane across a word of vertices.)
static __device__ __forceinline__ void emit_parent(const BParams &P, long long v, int u, unsigned long long bits)
{
    while (bits) {
        const int b = __ffsll((long long)bits) - 1;
        bits &= bits - 1;
        P.par[b][v] = u;
    }
}

// Level d+1 for the lanes `found` of this lane's vertex v: one store per lane
// b across the wavefront, so the 64 vertices of a word fill 256 contiguous
// bytes of root b's level array.  All lanes of the wavefront must be active.
static __device__ __forceinline__ void store_levels(const BParams &P, long long v, int d, unsigned long long found)
{
    if (!layer_stores_level(P, d + 1)) return;   // wave-uniform
    unsigned long long all = wave_or_u64(found);
    while (all) {
        const int b = __ffsll((long long)all) - 1;
        all &= all - 1;
        if ((found >> b) & 1ull) P.lvl[b][v] = d + 1;
    }
}

// Top-down edge u -> v for the lanes in m (u in their frontier, v not yet
// visited by them): the lanes' parent of v is the smallest such u, taken by
// an unsigned atomic minimum over the -1 the parents start from; the first
// edge to bring a lane stores its level (when the layer stores levels), the
// first to reach v at all marks v in the next frontier's bitmap.
static __device__ __forceinline__ void td_discover(const BParams &P, unsigned long long *next,
                                                   unsigned long long *unext, int v, int u, int d,
                                                   unsigned long long m)
{
    // plain reads first: next[v] only gains bits and parents only decrease,
    // so a stale read can only cost an unneeded atomic, never skip a needed one
    unsigned long long old = next[v];
    if ((old & m) != m) {
        old = atomicOr(&next[v], m);
        if (old == 0) atomicOr(&unext[v >> 6], 1ull << (v & 63));
    }
    const unsigned long long fresh = m & ~old;
    while (m) {
        const int b = __ffsll((long long)m) - 1;
        m &= m - 1;
        unsigned *pp = (unsigned *)&P.par[b][v];
        if ((fresh >> b) & 1ull) {
            atomicMin(pp, (unsigned)u);
            if (layer_stores_level(P, d + 1)) P.lvl[b][v] = d + 1;
        } else if (*pp > (unsigned)u) {
            atomicMin(pp, (unsigned)u);
        }
    }
}

// Bottom-up layer, rows longer than hub_deg.  Such a row is split into
// segments of 2^seg_log2 chunks of 2^hub_log2 entries, one wavefront per
// segment, so a long row is spread over many wavefronts; the segments are
// taken in the order of their number within the row (all rows' first
// segments, then the second ones, ...), so a row's earlier segments have
// mostly finished when its later ones start.  A wavefront scans
// its segment's chunks in ascending order, finding every pending lane's first
// hit (exclusive OR-scan over the lanes of each 64-entry step), and stops once
// all pending lanes have one.  Before each chunk it drops the lanes that the
// row's earlier segments have published as found: their hits are smaller ids,
// so the canonical parent of such a lane cannot lie in this segment.  (Masks
// left from earlier layers only hold lanes already visited at v, which are
// not pending.)  Across segments the smallest hit wins through an unsigned
// atomic minimum on the parent.  The segment's lanes are ORed into next[v];
// the pull kernel completes v.
static __device__ void push_bottom_up_hubs(const BParams &P, int d, long long gwave, long long nwaves)
{
    const int lane = __lane_id();
    const unsigned long long *front = fmask(P, d);
    const unsigned long long *ufront = P.ubm + (long long)(d % 3) * P.W;
    unsigned long long *next = fmask(P, d + 1);
    unsigned long long *unext = P.ubm + (long long)((d + 1) % 3) * P.W;
    const long long CH = 1ll << P.hub_log2;
    for (long long idx = gwave; idx < P.n_hseg; idx += nwaves) {
        const HSeg it = P.hseg[idx];
        const int v = it.v;
        unsigned long long rem = P.active & ~P.vis[v];
        if (!rem) continue;
        const int sj = it.seg;                              // segment number within the row
        const long long first = it.first;                   // found mask of the row's segment 0
        const long long sidx = first + sj;
        const long long rs = P.off[v], re = P.off[v + 1];
        const long long s = rs + ((long long)sj << (P.hub_log2 + P.seg_log2));
        const long long e = min(s + (CH << P.seg_log2), re);
        const bool publish = e < re;                        // later segments exist
        unsigned long long found = 0;
        for (long long cb = s; cb < e; cb += CH) {
            if (sj > 0) {
                unsigned long long x = 0;
                for (int t = lane; t < sj; t += 64) x |= ld_relaxed(&P.sfound[first + t]);
                rem &= ~wave_or_u64(x);
            }
            if (!rem) break;
            const long long ce = min(cb + CH, e);
            for (long long b = cb; b < ce && rem; b += 64) {
                const long long j = b + lane;
                int u = 0;
                unsigned long long f = 0;
                if (j < ce) {
                    u = P.col[j];
                    if (test_bit(ufront, u)) f = front[u] & rem;
                }
                if (!__ballot(f != 0)) continue;
                unsigned long long newb = f & ~wave_excl_or(f);
                while (newb) {
                    const int bb = __ffsll((long long)newb) - 1;
                    newb &= newb - 1;
                    atomicMin((unsigned *)&P.par[bb][v], (unsigned)u);
                    if (layer_stores_level(P, d + 1)) P.lvl[bb][v] = d + 1;
                }
                const unsigned long long all = wave_or_u64(f);
                rem &= ~all;
                found |= all;
            }
            if (publish && found && lane == 0)
                __hip_atomic_store(&P.sfound[sidx], found, __ATOMIC_RELAXED, AGENT);
        }
        if (found && lane == 0) {
            const unsigned long long old = atomicOr(&next[v], found);
            if (old == 0) atomicOr(&unext[v >> 6], 1ull << (v & 63));
        }
    }
}

struct BView {
    int done;
    int pad;
    BLayerState S;
    long long c[6];
    int *lvl[kLanes];                    // the lanes' output arrays, from the device table
    int *par[kLanes];
};

// Thread 0 reads the control data once per block; `coherent` reads the
// counters at the device-coherent level (needed in the single-block finisher,
// whose own atomics may be newer than its L1).
static __device__ void load_view(const BParams &P, int parity, int d_hint, BView *view, bool coherent)
{
    if (threadIdx.x < kLanes) view->lvl[threadIdx.x] = P.lvl[threadIdx.x];
    else if (threadIdx.x < 2 * kLanes) view->par[threadIdx.x - kLanes] = P.par[threadIdx.x - kLanes];
    if (threadIdx.x == 0) {
        BCtrl *C = P.ctrl;
        view->done = C->done;
        view->S = C->st[parity];
        BSlot &sl = C->slot[view->S.d % kSlots];
        for (int j = 0; j < 6; ++j) {
            long long a = 0;
            for (int k = 0; k < kSub; ++k) a += (long long)(coherent ? ld_relaxed(&sl.c[k][j]) : sl.c[k][j]);
            view->c[j] = a;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Push (top-down) for layer d.  Returns false when the batch is complete.
static __device__ bool batch_push(const BParams &Pin, int parity, int d_hint, long long gwave,
                                  long long nwaves, bool leader, BView *view, bool coherent)
{
    load_view(Pin, parity, d_hint, view, coherent);
    if (view->done) return false;
    BParams P = Pin;
    P.lvl = view->lvl;
    P.par = view->par;
    BCtrl *C = P.ctrl;
    const int d = view->S.d;
    if (d_hint >= 0 && d != d_hint) {
        if (leader) atomicOr((unsigned *)&C->status, 16u);
        return false;
    }
    const long long pairs = view->c[0];
    const long long m_u = view->S.m_u - view->c[3];
    if (pairs == 0 || d > P.n) {
        if (leader) {
            C->nlayers = d;
            C->pairs = view->S.pairs;
            C->pairs_deg = view->S.pairs_deg;
            C->done = d > P.n ? 2 : 1;
        }
        return false;
    }
    if (bdecide(P, view->S.dir_prev, view->c[1], view->c[2], m_u) != DIR_TD) {
        push_bottom_up_hubs(P, d, gwave, nwaves);
        return true;
    }

    const int lane = __lane_id();
    const unsigned long long *front = fmask(P, d);
    unsigned long long *next = fmask(P, d + 1);
    const unsigned long long *ufront = P.ubm + (long long)(d % 3) * P.W;
    unsigned long long *unext = P.ubm + (long long)((d + 1) % 3) * P.W;
    const int G = P.wpg_td;
    for (long long base = gwave * G; base < P.W; base += nwaves * G) {
        const long long myw = base + lane;
        const unsigned long long fwl = (lane < G && myw < P.W) ? ufront[myw] : 0ull;
        const int cnt = __popcll(fwl);
        const int cincl = wave_incl_scan32(cnt);
        const int cex = cincl - cnt;
        const int V = __builtin_amdgcn_readlane(cincl, 63);
        for (int vr = 0; vr < V; vr += 64) {
            const int vi = vr + lane;
            const bool vok = vi < V;
            const int l = lane_search(cex, vok ? vi : 0);
            const unsigned long long fw = (unsigned long long)__shfl((long long)fwl, l);
            const int kth = vi - __shfl(cex, l);
            int u = 0, dl = 0;
            long long sl = 0;
            unsigned long long fu = 0;
            if (vok) {
                u = (int)(((base + l) << 6) + select_bit(fw, kth));
                if ((unsigned)u >= (unsigned)P.n) {
                    atomicOr((unsigned *)&C->status, 8u);
                    u = 0;
                }
                dl = P.deg[u];
                sl = P.off[u];
                fu = front[u];
                if (dl > P.hub_deg) dl = 0;      // through the hub table below
            }
            const int incl = wave_incl_scan32(dl);
            const int ex = incl - dl;
            const int E = __builtin_amdgcn_readlane(incl, 63);
            for (int r0 = 0; r0 < E; r0 += 64) {
                const int idx = r0 + lane;
                const int lo = lane_search(ex, idx < E ? idx : 0);
                const long long j = __shfl(sl, lo) + (idx - __shfl(ex, lo));
                const unsigned long long fq = (unsigned long long)__shfl((long long)fu, lo);
                const int uq = __shfl(u, lo);
                if (idx < E) {
                    if ((unsigned long long)j >= (unsigned long long)P.nnz) {
                        atomicOr((unsigned *)&C->status, 4u);
                    } else {
                        const int v = P.col[j];
                        const unsigned long long m = fq & ~P.vis[v];
                        if (m) td_discover(P, next, unext, v, uq, d, m);
                    }
                }
            }
        }
    }
    if (view->c[4] > 0) {
        const long long CH = 1ll << P.hub_log2;
        for (long long b0 = gwave; b0 < P.n_hub; b0 += nwaves * 64) {
            const long long idx = b0 + (long long)lane * nwaves;
            Item it{-1, 0};
            if (idx < P.n_hub) it = P.hub[idx];
            const bool hit = it.u >= 0 && test_bit(ufront, it.u);
            unsigned long long m = __ballot(hit);
            while (m) {
                const int kk = __ffsll((long long)m) - 1;
                m &= m - 1;
                const int uh = __builtin_amdgcn_readlane(it.u, kk);
                const int ch = __builtin_amdgcn_readlane(it.chunk, kk);
                const unsigned long long fu = front[uh];
                const long long s = P.off[uh] + ((long long)ch << P.hub_log2);
                const long long e = min(s + CH, P.off[uh + 1]);
                for (long long j = s + lane; j < e; j += 64) {
                    const int v = P.col[j];
                    const unsigned long long mm = fu & ~P.vis[v];
                    if (mm) td_discover(P, next, unext, v, uh, d, mm);
                }
            }
        }
    }
    return true;
}

// ---------------------------------------------------------------------------
// Per-vertex bookkeeping once the lanes `found` reached v at level d+1.
static __device__ __forceinline__ void account(const BParams &P, unsigned long long vm, unsigned long long found,
                                               int dg, unsigned long long *cnt)
{
    const unsigned long long np = (unsigned long long)__popcll(found);
    cnt[0] += np;
    cnt[1] += 1;
    cnt[2] += (unsigned long long)dg;
    cnt[3] += ((vm | found) == P.active) ? (unsigned long long)dg : 0ull;
    cnt[4] += dg > P.hub_deg;
    cnt[5] += np * (unsigned long long)dg;
}

// After a top-down push: the vertices marked in unext are F_{d+1}; fold their
// masks into vis and count them.  The marked vertices of a task of 64 words
// are laid out over the lanes.
static __device__ void pull_after_push(const BParams &P, const unsigned long long *next,
                                       const unsigned long long *unext, long long gwave, long long nwaves,
                                       unsigned long long *cnt)
{
    const int lane = __lane_id();
    for (long long base = gwave * 64; base < P.W; base += nwaves * 64) {
        const long long myw = base + lane;
        const unsigned long long uw = myw < P.W ? unext[myw] : 0ull;
        const int c = __popcll(uw);
        const int cincl = wave_incl_scan32(c);
        const int cex = cincl - c;
        const int V = __builtin_amdgcn_readlane(cincl, 63);
        for (int vr = 0; vr < V; vr += 64) {
            const int vi = vr + lane;
            const int l = lane_search(cex, vi < V ? vi : 0);
            const unsigned long long wbits = (unsigned long long)__shfl((long long)uw, l);
            const int kth = vi - __shfl(cex, l);
            if (vi < V) {
                const long long v = ((base + l) << 6) + select_bit(wbits, kth);
                const unsigned long long found = next[v];
                const unsigned long long vm = P.vis[v];
                P.vis[v] = vm | found;
                account(P, vm, found, P.deg[v], cnt);
            }
        }
    }
}

// Bottom-up (Algorithm 2 on masks): every vertex with lanes still unvisited
// scans its ascending row; the first u whose frontier mask holds lane b is
// lane b's parent.  A neighbour's 8-byte mask is only loaded when the bitmap
// of the union frontier (n/8 bytes, cache-resident) marks it.  Rows up to 32
// entries are scanned by their own lane, four entries per step; rows up to
// hub_deg by the whole wavefront, 64 entries per step, the first occurrence
// of each lane in a step coming from an exclusive OR-scan over the lanes;
// longer rows were scanned in chunks by the push kernel.
// STAGED: for a word's 64 vertices the position of lane b's parent within
// the row is kept in LDS (spos, [lane b][vertex] bytes = 4 KB per wavefront;
// rows handled here have at most hub_deg <= 256 entries), and the parents
// and levels are then stored per root b as 256-byte runs, instead of one
// scattered 4-byte store per (root, vertex).
template <bool STAGED>
static __device__ void pull_bottom_up(const BParams &P, int d, const unsigned long long *front,
                                      const unsigned long long *ufront, unsigned long long *next,
                                      unsigned long long *unext, long long gwave, long long nwaves,
                                      unsigned long long *cnt, unsigned char *spos)
{
    const int lane = __lane_id();
    const int G = P.wpg;
    for (long long base = gwave * G; base < P.W; base += nwaves * G) {
        for (int wi = 0; wi < G; ++wi) {
            const long long w = base + wi;
            if (w >= P.W) break;
            const long long v = (w << 6) + lane;
            unsigned long long vm = P.active, need = 0;
            if (v < P.n) {
                vm = P.vis[v];
                need = P.active & ~vm;
            }
            if (!__ballot(need != 0)) continue;
            const int dg = need ? P.deg[v] : 0;
            long long s = 0;
            unsigned long long found = 0;
            const bool hub = dg > P.hub_deg;
            if (hub) {
                found = next[v];        // from the chunk scans of this layer
                need = 0;
            }
            if (need && dg > 0) s = P.off[v];
            if (need && dg > 0 && dg <= 32) {
                const long long e = s + dg;
                unsigned long long rem = need;
                for (long long j0 = s; j0 < e && rem; j0 += 4) {
                    int uq[4];
                    unsigned long long fq[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) uq[q] = j0 + q < e ? P.col[j0 + q] : -1;
                    bool in[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) in[q] = uq[q] >= 0 && test_bit(ufront, uq[q]);
#pragma unroll
                    for (int q = 0; q < 4; ++q) fq[q] = in[q] ? front[uq[q]] : 0ull;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const unsigned long long f = fq[q] & rem;
                        if (f) {
                            if (STAGED) {
                                unsigned long long bits = f;
                                while (bits) {
                                    const int b = __ffsll((long long)bits) - 1;
                                    bits &= bits - 1;
                                    spos[b * 64 + lane] = (unsigned char)(j0 + q - s);
                                }
                            } else {
                                emit_parent(P, v, uq[q], f);
                            }
                            found |= f;
                            rem &= ~f;
                        }
                    }
                }
            }
            unsigned long long longm = __ballot(need != 0 && dg > 32);   // up to hub_deg
            while (longm) {
                const int k = __ffsll((long long)longm) - 1;
                longm &= longm - 1;
                const long long vk = bcast64(v, k);
                const long long sk = bcast64(s, k);
                const long long ek = sk + __builtin_amdgcn_readlane(dg, k);
                unsigned long long remk = bcast_u64(need, k);
                unsigned long long foundk = 0;
                for (long long b = sk; b < ek && remk; b += 64) {
                    const long long j = b + lane;
                    int u = 0;
                    unsigned long long f = 0;
                    if (j < ek) {
                        u = P.col[j];
                        if (test_bit(ufront, u)) f = front[u] & remk;
                    }
                    if (!__ballot(f != 0)) continue;
                    unsigned long long newb = f & ~wave_excl_or(f);
                    if (STAGED) {
                        while (newb) {
                            const int bb = __ffsll((long long)newb) - 1;
                            newb &= newb - 1;
                            spos[bb * 64 + k] = (unsigned char)(j - sk);
                        }
                    } else if (newb) {
                        emit_parent(P, vk, u, newb);
                    }
                    const unsigned long long all = wave_or_u64(f);
                    remk &= ~all;
                    foundk |= all;
                }
                if (lane == k) found |= foundk;
            }
            const unsigned long long mine = hub ? 0ull : found;
            if (STAGED) {
                // LDS writes of other lanes above must be complete before the reads
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                unsigned long long all = wave_or_u64(mine);
                while (all) {
                    const int b = __ffsll((long long)all) - 1;
                    all &= all - 1;
                    if ((mine >> b) & 1ull) {
                        P.par[b][v] = P.col[s + spos[b * 64 + lane]];
                        if (layer_stores_level(P, d + 1)) P.lvl[b][v] = d + 1;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
            } else {
                store_levels(P, v, d, mine);
            }
            if (found) {
                if (!hub) next[v] = found;
                P.vis[v] = vm | found;
                account(P, vm, found, dg, cnt);
            }
            const unsigned long long um = __ballot(found != 0);
            if (lane == 0 && um) unext[w] = um;
        }
    }
}

// Pull for layer d: F_{d+1} into vis, its counters, and the buffers of F_{d-1}
// cleared for reuse as `next` of layer d+1.
template <bool STAGED>
static __device__ void batch_pull(const BParams &Pin, int parity, int d_hint, long long gwave,
                                  long long nwaves, bool leader, BView *view, unsigned long long *s_red,
                                  int nwaves_block, bool coherent, unsigned char *spos)
{
    load_view(Pin, parity, d_hint, view, coherent);
    if (view->done) return;
    BParams P = Pin;
    P.lvl = view->lvl;
    P.par = view->par;
    BCtrl *C = P.ctrl;
    const int d = view->S.d;
    if (d_hint >= 0 && d != d_hint) return;
    // the same decision as the push kernel of this layer, from the same data
    const long long m_u = view->S.m_u - view->c[3];
    const int cur = bdecide(P, view->S.dir_prev, view->c[1], view->c[2], m_u);
    const int lane = __lane_id();
    const unsigned long long *front = fmask(P, d);
    unsigned long long *next = fmask(P, d + 1);
    // F_{d-1}'s masks are cleared for reuse only in the rotating slots; a
    // kept slot waits for the level pass
    unsigned long long *spare = d - 1 >= P.hist ? fmask(P, d - 1) : nullptr;
    unsigned long long *unext = P.ubm + (long long)((d + 1) % 3) * P.W;
    unsigned long long *uspare = P.ubm + (long long)((d + 2) % 3) * P.W;
    unsigned long long cnt[6] = {0, 0, 0, 0, 0, 0};
    if (cur == DIR_TD)
        pull_after_push(P, next, unext, gwave, nwaves, cnt);
    else
        pull_bottom_up<STAGED>(P, d, front, P.ubm + (long long)(d % 3) * P.W, next, unext, gwave, nwaves, cnt,
                               spos);
    // F_{d-1}: its masks are nonzero exactly at the vertices its bitmap marks;
    // the bitmap itself always rotates
    for (long long base = gwave * 64; base < P.W; base += nwaves * 64) {
        const long long myw = base + lane;
        const unsigned long long sw = myw < P.W ? uspare[myw] : 0ull;
        unsigned long long todo = __ballot(sw != 0);
        while (todo) {
            const int k = __ffsll((long long)todo) - 1;
            todo &= todo - 1;
            const unsigned long long bits = bcast_u64(sw, k);
            if (spare && ((bits >> lane) & 1ull)) spare[((base + k) << 6) + lane] = 0ull;
        }
        if (sw) uspare[myw] = 0ull;
    }
    if (leader) {
        BLayerState Nx = view->S;
        Nx.d = d + 1;
        Nx.dir_prev = cur;
        Nx.m_u = m_u;
        Nx.pairs = view->S.pairs + view->c[0];
        Nx.pairs_deg = view->S.pairs_deg + view->c[5];
        C->st[parity ^ 1] = Nx;
        C->parity = parity ^ 1;
        BSlot *Z = &C->slot[(d + 2) % kSlots];
        for (int k = 0; k < kSub; ++k)
            for (int j = 0; j < 6; ++j) Z->c[k][j] = 0;
        if (d < P.trace_cap) {
            LayerRec r;
            r.dir = cur;
            r.pad = 0;
            r.n_f = view->c[1];
            r.m_f = view->c[2];
            r.m_u = m_u;
            r.v_u = -1;
            P.trace[d] = r;
        }
    }
    // counters of F_{d+1}
    const int wib = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const unsigned long long t = wave_sum_u64(cnt[j]);
        if (lane == 0) s_red[6 * wib + j] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        BSlot &sl = C->slot[(d + 1) % kSlots];
        unsigned long long *sub = sl.c[blockIdx.x % kSub];
        for (int j = 0; j < 6; ++j) {
            unsigned long long a = 0;
            for (int i = 0; i < nwaves_block; ++i) a += s_red[6 * i + j];
            if (a) atomicAdd(&sub[j], a);
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Grid (x, k + 1): row y < k fills lane y's parents with -1 (the start of
// their atomic minima; the levels are all stored by the level pass or the
// layers); row k clears the rotating masks and bitmaps, stores the output
// table and resets the control block.  The kept slots are already clear:
// a new workspace starts zeroed, and every level pass clears what it read.
__global__ void __launch_bounds__(kBlock) bfs_batch_init_kernel(BParams P, LanePtrs out)
{
    const long long gt = (long long)blockIdx.x * kBlock + threadIdx.x;
    const long long nt = (long long)gridDim.x * kBlock;
    const int y = blockIdx.y;
    if (y < P.k) {
        int *pa = out.parent[y];
        const bool vec = (((unsigned long long)pa) & 15ull) == 0;
        const long long n4 = vec ? (P.n >> 2) : 0;
        // non-temporal 16-byte stores: the 4·k·n bytes of -1 are not read
        // again by this kernel, and keeping them out of L2 leaves more of it
        // to the layers
        typedef int v4i __attribute__((ext_vector_type(4)));
        const v4i m1 = {-1, -1, -1, -1};
        for (long long i = gt; i < n4; i += nt) __builtin_nontemporal_store(m1, (v4i *)pa + i);
        for (long long i = (n4 << 2) + gt; i < P.n; i += nt) pa[i] = -1;
        return;
    }
    for (long long v = gt; v < P.n; v += nt) {
        // vertices without edges count as visited in every lane: they are
        // never reached (a root among them is seeded separately)
        P.vis[v] = test_bit(P.iso, (int)v) ? P.active : 0ull;
        // every layer clears only what it set, so the three rotating slots
        // start empty
        unsigned long long *rot = P.fm + (long long)P.hist * P.n;
        rot[v] = 0ull;
        rot[P.n + v] = 0ull;
        rot[2 * P.n + v] = 0ull;
    }
    for (long long w = gt; w < P.W; w += nt) {
        P.ubm[w] = 0ull;
        P.ubm[P.W + w] = 0ull;
        P.ubm[2 * P.W + w] = 0ull;
    }
    for (long long i = gt; i < P.n_hseg; i += nt) P.sfound[i] = 0ull;
    if (gt < kLanes) {
        const_cast<int **>(P.lvl)[gt] = gt < P.k ? out.level[gt] : nullptr;
        const_cast<int **>(P.par)[gt] = gt < P.k ? out.parent[gt] : nullptr;
    }
    if (gt == 0) {
        BCtrl *C = P.ctrl;
        C->done = 0;
        C->nlayers = 0;
        C->parity = 0;
        C->status = 0;
        C->async_run = P.async_run;
        C->fail_injected = P.fail_injected;
        C->pairs = 0;
        C->pairs_deg = 0;
        BLayerState S;
        S.d = 0;
        S.dir_prev = DIR_TD;
        S.m_u = P.nnz;
        S.pairs = 0;
        S.pairs_deg = 0;
        for (int i = 0; i < 4; ++i) S.pad[i] = 0;
        C->st[0] = S;
        C->st[1] = S;
        for (int k = 0; k < kSlots; ++k)
            for (int j = 0; j < kSub; ++j)
                for (int c = 0; c < 8; ++c) C->slot[k].c[j][c] = 0;
    }
}

// One wavefront: the roots' entries, masks and the counters of F_0.
__global__ void __launch_bounds__(64) bfs_batch_seed_kernel(BParams P, RootSet R)
{
    const int lane = threadIdx.x;
    const bool on = lane < P.k;
    const int r = on ? R.r[lane] : -1;
    unsigned long long mask = 0;
    bool first = on;
    for (int b = 0; b < kLanes; ++b) {
        const int rb = __shfl(r, b);
        if (on && b < P.k && rb == r) {
            mask |= 1ull << b;
            if (b < lane) first = false;
        }
    }
    unsigned long long c1 = 0, c2 = 0, c3 = 0, c4 = 0, c5 = 0;
    if (on) {
        if (layer_stores_level(P, 0)) P.lvl[lane][r] = 0;
        P.par[lane][r] = r;
        c5 = (unsigned long long)P.deg[r];
    }
    if (first) {
        const unsigned long long vm = test_bit(P.iso, r) ? P.active : 0ull;
        fmask(P, 0)[r] = mask;
        P.vis[r] = vm | mask;
        atomicOr(&P.ubm[r >> 6], 1ull << (r & 63));
        const int dg = P.deg[r];
        c1 = 1;
        c2 = (unsigned long long)dg;
        c3 = (mask == P.active && vm != P.active) ? (unsigned long long)dg : 0ull;
        c4 = dg > P.hub_deg;
    }
    c1 = wave_sum_u64(c1);
    c2 = wave_sum_u64(c2);
    c3 = wave_sum_u64(c3);
    c4 = wave_sum_u64(c4);
    c5 = wave_sum_u64(c5);
    if (lane == 0) {
        BSlot &sl = P.ctrl->slot[0];
        sl.c[0][0] = (unsigned long long)P.k;
        sl.c[0][1] = c1;
        sl.c[0][2] = c2;
        sl.c[0][3] = c3;
        sl.c[0][4] = c4;
        sl.c[0][5] = c5;
    }
}

__global__ void __launch_bounds__(kBlock) bfs_batch_push_kernel(BParams P, int layer)
{
    __shared__ BView view;
    const long long gwave = (long long)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const long long nwaves = (long long)gridDim.x * kWavesPerBlock;
    batch_push(P, layer & 1, layer, gwave, nwaves, blockIdx.x == 0 && threadIdx.x == 0, &view, false);
}

__global__ void __launch_bounds__(kPullWaves * 64) bfs_batch_pull_kernel(BParams P, int layer)
{
    __shared__ BView view;
    __shared__ unsigned long long s_red[6 * kPullWaves];
    __shared__ unsigned char s_pos[kPullWaves][64 * 64];
    const int wib = threadIdx.x >> 6;
    const long long gwave = (long long)blockIdx.x * kPullWaves + wib;
    const long long nwaves = (long long)gridDim.x * kPullWaves;
    batch_pull<true>(P, layer & 1, layer, gwave, nwaves, blockIdx.x == 0 && threadIdx.x == 0, &view, s_red,
                     kPullWaves, false, s_pos[wib]);
}

// One block runs whatever layers remain, with block barriers between phases.
__global__ void __launch_bounds__(kFinishBlock) bfs_batch_finish_kernel(BParams P)
{
    __shared__ BView view;
    __shared__ unsigned long long s_red[6 * (kFinishBlock / 64)];
    __shared__ int s_parity;
    const long long gwave = threadIdx.x >> 6;
    const long long nwaves = kFinishBlock / 64;
    for (;;) {
        if (threadIdx.x == 0) s_parity = P.ctrl->parity;
        __syncthreads();
        const int parity = s_parity;
        __syncthreads();
        if (!batch_push(P, parity, -1, gwave, nwaves, threadIdx.x == 0, &view, true)) break;
        __syncthreads();
        batch_pull<false>(P, parity, -1, gwave, nwaves, threadIdx.x == 0, &view, s_red, kFinishBlock / 64, true,
                          nullptr);
        __syncthreads();
    }
    __syncthreads();
    if (threadIdx.x == 0) record_failure(P.ctrl);
}

// Level pass, after the finisher: lane b's level of v for every level below
// P.hist, read from the kept masks (bit b of v's mask in F_d: root b reached
// v at level d), and -1 where root b never reached v; levels from P.hist on
// were stored by their layers and are left alone.  One wavefront per bitmap
// word, lane i on vertex 64w + i, so each store of root b's levels covers 256
// contiguous bytes.  The per-lane level comes from four bit-slices of the
// kept masks (slice j: the lanes whose level has bit j set).  The kept masks
// read are cleared for the next batch: those of the levels the traversal
// reached, or all of them after a failed traversal.
__global__ void __launch_bounds__(kBlock) bfs_batch_levels_kernel(BParams P)
{
    const int lane = __lane_id();
    const long long gwave = (long long)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const long long nwaves = (long long)gridDim.x * kWavesPerBlock;
    const BCtrl *C = P.ctrl;
    const bool ok = C->done == 1 && C->status == 0;
    const int D = ok ? min(P.hist, C->nlayers) : P.hist;
    for (long long w = gwave; w < P.W; w += nwaves) {
        const long long v = (w << 6) + lane;
        const bool in = v < P.n;
        // all kept masks of v in flight together
        unsigned long long h[kBatchHist];
#pragma unroll
        for (int d = 0; d < kBatchHist; ++d) h[d] = (d < D && in) ? P.fm[(long long)d * P.n + v] : 0ull;
        const unsigned long long vis = in ? P.vis[v] : 0ull;
        const bool iso = in && test_bit(P.iso, (int)v);
        unsigned long long sl[4] = {0ull, 0ull, 0ull, 0ull};
        unsigned long long kept = 0;          // lanes whose level of v is below P.hist
#pragma unroll
        for (int d = 0; d < kBatchHist; ++d) {
            kept |= h[d];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if ((d >> j) & 1) sl[j] |= h[d];
        }
#pragma unroll
        for (int d = 0; d < kBatchHist; ++d)
            if (h[d]) P.fm[(long long)d * P.n + v] = 0ull;
        // the lanes that reached v: those that visited it, except that a
        // vertex without edges counts as visited in every lane from the start
        // and is reached only as a root (level 0)
        const unsigned long long reached = iso ? kept : vis;
        // stored here: the kept levels and -1 for the lanes that never reached v
        const unsigned long long mine = in ? (kept | ~reached) : 0ull;
        if (!__ballot(mine != 0)) continue;
        for (int b = 0; b < P.k; ++b) {
            if (!((mine >> b) & 1ull)) continue;
            int lev = -1;
            if ((kept >> b) & 1ull)
                lev = (int)((sl[0] >> b) & 1ull) | (int)(((sl[1] >> b) & 1ull) << 1) |
                      (int)(((sl[2] >> b) & 1ull) << 2) | (int)(((sl[3] >> b) & 1ull) << 3);
            __builtin_nontemporal_store(lev, &P.lvl[b][v]);
        }
    }
}

hipError_t launch_batch_init(const BParams &p, const LanePtrs &out, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(bfs_batch_init_kernel, dim3(grid, p.k + 1), dim3(kBlock), 0, s, p, out);
    return hipGetLastError();
}

hipError_t launch_batch_seed(const BParams &p, const RootSet &roots, hipStream_t s)
{
    hipLaunchKernelGGL(bfs_batch_seed_kernel, dim3(1), dim3(64), 0, s, p, roots);
    return hipGetLastError();
}

hipError_t launch_batch_push(const BParams &p, int layer, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(bfs_batch_push_kernel, dim3(grid), dim3(kBlock), 0, s, p, layer);
    return hipGetLastError();
}

hipError_t launch_batch_pull(const BParams &p, int layer, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(bfs_batch_pull_kernel, dim3(grid), dim3(kPullWaves * 64), 0, s, p, layer);
    return hipGetLastError();
}

hipError_t launch_batch_finish(const BParams &p, hipStream_t s)
{
    hipLaunchKernelGGL(bfs_batch_finish_kernel, dim3(1), dim3(kFinishBlock), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_batch_levels(const BParams &p, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(bfs_batch_levels_kernel, dim3(grid), dim3(kBlock), 0, s, p);
    return hipGetLastError();
}

void *kernel_ptr_batch(int which)
{
    switch (which) {
    case BK_INIT: return (void *)bfs_batch_init_kernel;
    case BK_SEED: return (void *)bfs_batch_seed_kernel;
    case BK_PUSH: return (void *)bfs_batch_push_kernel;
    case BK_PULL: return (void *)bfs_batch_pull_kernel;
    case BK_LEVELS: return (void *)bfs_batch_levels_kernel;
    default: return (void *)bfs_batch_finish_kernel;
    }
}

int batch_blocks_per_cu()
{
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, bfs_batch_push_kernel, kBlock, 0) != hipSuccess) return -1;
    return b;
}

int batch_pull_blocks_per_cu()
{
    int a = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, bfs_batch_pull_kernel, kPullWaves * 64, 0) != hipSuccess)
        return -1;
    return a;
}

}  // namespace hybfs
