/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, serial, obviously correct implementation of what the hybrid
 * (direction-optimising) breadth-first search computes.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the GPU
 * library neither links nor calls it, and it shares no code with the GPU path.
 *
 * What is computed (paper Section 4: layers, frontier, output queue, visited
 * set and predecessor array P; Algorithms 1-3):
 *   level[v]  = hop distance from the root (the index of v's layer), or -1
 *               when v is not reachable.  Layers are unique whatever order a
 *               layer-synchronous traversal uses inside a layer.
 *   parent[v] = the predecessor in the BFS tree.  The paper notes that a
 *               parallel traversal may return different valid trees from run to
 *               run (Section 7.1); this build fixes the tree to the canonical
 *               one: parent[root] = root, and for every other reached v the
 *               smallest vertex id among v's neighbours one layer closer to the
 *               root.  Unreached vertices get parent -1.
 * Both outputs are a function of the graph and the root only, so any schedule
 * of top-down / bottom-up layers must reproduce them byte for byte.
 *
 * The per-layer counters follow Section 4's online heuristic inputs: the
 * number of vertices in the frontier (v_f), the edges to check from the
 * frontier (e_f = sum of frontier degrees) and the edges of the not yet
 * visited vertices (e_u); the switch functions f and g are evaluated as the
 * state machine that reproduces Table 2.
 */
#include <stdint.h>
#include <stdlib.h>

/* ---- levels: FIFO breadth-first search (Section 4, layer-synchronous BFS) ---- */
int oracle_bfs_levels(int64_t n, const int64_t *off, const int32_t *col,
                      int32_t root, int32_t *level)
{
    if (n <= 0 || root < 0 || root >= n) return -1;
    int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!queue) return -2;
    for (int64_t v = 0; v < n; ++v) level[v] = -1;
    int64_t head = 0, tail = 0;
    level[root] = 0;
    queue[tail++] = root;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int64_t j = off[u]; j < off[u + 1]; ++j) {
            int32_t w = col[j];
            if (level[w] == -1) {
                level[w] = level[u] + 1;
                queue[tail++] = w;
            }
        }
    }
    free(queue);
    return 0;
}

/* ---- canonical parents: the smallest neighbour id one layer up ----
 * Scans the whole adjacency list; does not rely on rows being sorted. */
int oracle_canonical_parents(int64_t n, const int64_t *off, const int32_t *col,
                             int32_t root, const int32_t *level, int32_t *parent)
{
    if (n <= 0 || root < 0 || root >= n) return -1;
    for (int64_t v = 0; v < n; ++v) {
        parent[v] = -1;
        if (level[v] <= 0) continue;
        int32_t best = -1;
        for (int64_t j = off[v]; j < off[v + 1]; ++j) {
            int32_t u = col[j];
            if (level[u] == level[v] - 1 && (best == -1 || u < best)) best = u;
        }
        parent[v] = best;
    }
    parent[root] = root;
    return 0;
}

int oracle_bfs(int64_t n, const int64_t *off, const int32_t *col, int32_t root,
               int32_t *level, int32_t *parent)
{
    int rc = oracle_bfs_levels(n, off, col, root, level);
    if (rc) return rc;
    return oracle_canonical_parents(n, off, col, root, level, parent);
}

/* ---- per-layer replay of the heuristic's inputs (Section 4, Algorithm 3) ----
 * For d = 0 .. L-1 (L = deepest level + 1):
 *   n_f[d] = |F_d|, F_d = {v : level[v] == d}          (v_f in the paper)
 *   m_f[d] = sum of deg(v) over F_d                       (e_f)
 *   m_u[d] = sum of deg(v) over {v : level[v] > d or -1}  (e_u, edges of the
 *            vertices not in layers 0..d)
 *   v_u[d] = |{v : level[v] > d or -1}|                  (the vertex count that
 *            Table 2's "e_u" column actually holds)
 * Returns L, or -1 if L exceeds cap (arrays then hold the first cap layers). */
int64_t oracle_layer_replay(int64_t n, const int64_t *off, const int32_t *level,
                            int64_t cap, int64_t *n_f, int64_t *m_f,
                            int64_t *m_u, int64_t *v_u)
{
    int32_t maxl = -1;
    for (int64_t v = 0; v < n; ++v)
        if (level[v] > maxl) maxl = level[v];
    int64_t L = (int64_t)maxl + 1;
    int64_t upto = L < cap ? L : cap;
    for (int64_t d = 0; d < upto; ++d) {
        int64_t nf = 0, mf = 0, mu = 0, vu = 0;
        for (int64_t v = 0; v < n; ++v) {
            int64_t deg = off[v + 1] - off[v];
            if (level[v] == d) { nf += 1; mf += deg; }
            if (level[v] > d || level[v] == -1) { mu += deg; vu += 1; }
        }
        n_f[d] = nf; m_f[d] = mf; m_u[d] = mu; v_u[d] = vu;
    }
    return L <= cap ? L : -1;
}

/* ---- direction of each layer (Algorithm 3 read as a state machine) ----
 * rule 0 (edge counts, Beamer et al.): from top-down switch to bottom-up when
 *        m_f * alpha > m_u; from bottom-up switch back when n_f * beta < n.
 * rule 1 (Table 2 reading): f = floor(v_u / 1024), g = floor(n / 64); from
 *        top-down switch when n_f > f; from bottom-up switch back when n_f < g.
 * rule 2: every layer top-down.  rule 3: every layer bottom-up.
 * The traversal starts in top-down (Algorithm 3 initialises topdown=true) and
 * the test is applied before each layer, including the first.
 * dir[d] = 0 for top-down, 1 for bottom-up. */
int oracle_direction_trace(int rule, int64_t alpha, int64_t beta, int64_t n,
                           int64_t L, const int64_t *n_f, const int64_t *m_f,
                           const int64_t *m_u, const int64_t *v_u, int32_t *dir)
{
    int32_t cur = 0;
    for (int64_t d = 0; d < L; ++d) {
        if (rule == 2) cur = 0;
        else if (rule == 3) cur = 1;
        else if (rule == 0) {
            if (cur == 0 && m_f[d] * alpha > m_u[d]) cur = 1;
            else if (cur == 1 && n_f[d] * beta < n) cur = 0;
        } else if (rule == 1) {
            int64_t f = v_u[d] / 1024, g = n / 64;
            if (cur == 0 && n_f[d] > f) cur = 1;
            else if (cur == 1 && n_f[d] < g) cur = 0;
        } else {
            return -1;
        }
        dir[d] = cur;
    }
    return 0;
}

/* ---- traversed edges: directed CSR entries of the reached vertices ----
 * (the TEPS numerator is half of this for a symmetric graph; Section 6.3) */
int64_t oracle_reached_degree_sum(int64_t n, const int64_t *off, const int32_t *level)
{
    int64_t s = 0;
    for (int64_t v = 0; v < n; ++v)
        if (level[v] >= 0) s += off[v + 1] - off[v];
    return s;
}

/* ---- bottom-up probe count of one layer ----
 * For every v with deg(v) > 0 that is not in layers 0..d: the number of
 * adjacency entries a bottom-up step (Algorithm 2) reads before it stops,
 * scanning in stored (ascending) order: 1 + the index of the first neighbour in
 * F_d, or deg(v) if there is none.  Returns the sum and the vertex count. */
int64_t oracle_bottom_up_probes(int64_t n, const int64_t *off, const int32_t *col,
                                const int32_t *level, int32_t d, int64_t *n_candidates)
{
    int64_t sum = 0, cnt = 0;
    for (int64_t v = 0; v < n; ++v) {
        int64_t deg = off[v + 1] - off[v];
        if (deg == 0) continue;
        if (!(level[v] > d || level[v] == -1)) continue;
        cnt += 1;
        int64_t s = deg;
        for (int64_t j = off[v]; j < off[v + 1]; ++j) {
            if (level[col[j]] == d) { s = j - off[v] + 1; break; }
        }
        sum += s;
    }
    if (n_candidates) *n_candidates = cnt;
    return sum;
}
