"""Independent checks used to pin the oracle and to validate GPU outputs.

None of this calls the oracle: the brute-force distances use Floyd-Warshall
on a dense matrix, components use union-find, and the closed forms are
derived by hand for each graph family.
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------- brute force
def floyd_warshall(g) -> np.ndarray:
    """All-pairs hop distances (inf where unreachable) from a dense matrix."""
    n = g.n
    INF = np.inf
    D = np.full((n, n), INF)
    np.fill_diagonal(D, 0.0)
    for v in range(n):
        for j in range(g.off[v], g.off[v + 1]):
            u = int(g.col[j])
            if u != v:
                D[v, u] = 1.0
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    return D


def brute_force_bfs(g, root: int, D: np.ndarray | None = None):
    """Levels from the distance matrix; parent = smallest-id adjacent vertex one
    hop closer, found from a dense adjacency matrix."""
    if D is None:
        D = floyd_warshall(g)
    n = g.n
    A = np.zeros((n, n), dtype=bool)
    for v in range(n):
        A[v, g.col[g.off[v]:g.off[v + 1]]] = True
    dist = D[root]
    level = np.where(np.isinf(dist), -1, dist).astype(np.int32)
    parent = np.full(n, -1, dtype=np.int32)
    for v in range(n):
        if v == root:
            parent[v] = root
        elif level[v] > 0:
            cand = np.nonzero(A[v] & (dist == dist[v] - 1))[0]
            parent[v] = cand.min()
    return level, parent


# ---------------------------------------------------------------- invariants
def components(g) -> np.ndarray:
    """Connected-component label per vertex (union-find with path halving)."""
    parent = np.arange(g.n)

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    src = np.repeat(np.arange(g.n), np.diff(g.off))
    for a, b in zip(src.tolist(), g.col.tolist()):
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)
    return np.array([find(x) for x in range(g.n)])


def check_bfs_invariants(g, root: int, level: np.ndarray, parent: np.ndarray,
                         comp: np.ndarray | None = None, canonical: bool = True) -> None:
    """Graph500-style validation plus canonical-parent and component checks.
    Vectorised over edges (O(n + nnz)); raises AssertionError on failure.
    canonical=False accepts any neighbour one layer closer as the parent."""
    n = g.n
    level = np.asarray(level)
    parent = np.asarray(parent)
    assert level.shape == (n,) and parent.shape == (n,)
    assert level[root] == 0 and parent[root] == root
    reached = level >= 0
    assert np.all(parent[~reached] == -1)
    assert np.all(level[reached & (np.arange(n) != root)] > 0)
    src = np.repeat(np.arange(n), np.diff(g.off))
    dst = g.col.astype(np.int64)
    # no edge joins a reached and an unreached vertex
    assert np.all(reached[src] == reached[dst])
    # edges between reached vertices span at most one layer
    both = reached[src] & reached[dst]
    assert np.all(np.abs(level[src[both]] - level[dst[both]]) <= 1)
    # tree edges: parent is adjacent and one layer closer
    others = np.nonzero(reached & (np.arange(n) != root))[0]
    if len(others):
        p = parent[others]
        assert np.all((p >= 0) & (p < n))
        assert np.all(level[p] == level[others] - 1)
        closer = both & (level[dst] == level[src] - 1)
        if canonical:
            # parent[v] is the minimum over neighbours one layer closer
            best = np.full(n, np.iinfo(np.int64).max)
            np.minimum.at(best, src[closer], dst[closer])
            assert np.all(best[others] == p)
        else:
            # (v, parent[v]) is an edge of the graph
            keys = np.sort(src[closer] * n + dst[closer])
            want = others.astype(np.int64) * n + p.astype(np.int64)
            pos = np.searchsorted(keys, want)
            assert np.all((pos < len(keys)) & (keys[np.minimum(pos, len(keys) - 1)] == want))
    # reached set equals the root's connected component
    if comp is not None:
        assert np.array_equal(reached, comp == comp[root])


# ---------------------------------------------------------------- closed forms
def path_expected(n: int, r: int):
    i = np.arange(n)
    level = np.abs(i - r).astype(np.int32)
    parent = np.where(i > r, i - 1, np.where(i < r, i + 1, r)).astype(np.int32)
    return level, parent


def cycle_expected(n: int, r: int):
    i = np.arange(n)
    k = (i - r) % n                      # steps going "up" from r
    level = np.minimum(k, n - k).astype(np.int32)
    parent = np.empty(n, dtype=np.int32)
    for v in range(n):
        if v == r:
            parent[v] = r
            continue
        cands = []
        if k[v] <= n - k[v]:             # reachable going up: predecessor v-1
            cands.append((v - 1) % n)
        if n - k[v] <= k[v]:             # reachable going down: successor v+1
            cands.append((v + 1) % n)
        parent[v] = min(cands)
    return level, parent


def grid_expected(rows: int, cols: int, r: int):
    n = rows * cols
    r0, c0 = divmod(r, cols)
    level = np.empty(n, dtype=np.int32)
    parent = np.empty(n, dtype=np.int32)
    for v in range(n):
        rv, cv = divmod(v, cols)
        level[v] = abs(rv - r0) + abs(cv - c0)
        if v == r:
            parent[v] = r
            continue
        cands = []
        if rv != r0:
            cands.append(v - cols if rv > r0 else v + cols)
        if cv != c0:
            cands.append(v - 1 if cv > c0 else v + 1)
        parent[v] = min(cands)
    return level, parent


def hypercube_expected(dim: int, r: int):
    """level = popcount(v xor r).  Closer neighbours flip one bit of v xor r;
    the smallest id clears the highest bit that v has set among them, else sets
    the lowest differing bit."""
    n = 1 << dim
    level = np.empty(n, dtype=np.int32)
    parent = np.empty(n, dtype=np.int32)
    for v in range(n):
        x = v ^ r
        level[v] = bin(x).count("1")
        if v == r:
            parent[v] = r
            continue
        down = v & x
        if down:
            b = down.bit_length() - 1
        else:
            b = (x & -x).bit_length() - 1
        parent[v] = v ^ (1 << b)
    return level, parent


def batch_union_replay(g, levels) -> dict:
    """Per-layer counters a batched traversal decides on, from the roots' level
    arrays (k x n): n_f and m_f over the union of the roots' frontiers F_d, and
    m_u = degree sum of the vertices that are not yet at a level <= d in every
    root's traversal."""
    lv = np.asarray(levels, dtype=np.int64).reshape(-1, g.n)
    deg = np.diff(np.asarray(g.off, dtype=np.int64))
    L = int(lv.max()) + 1 if lv.size else 0
    unreached = np.where(lv < 0, np.iinfo(np.int64).max, lv)
    done_at = unreached.max(axis=0)        # layer after which v is visited in every root
    out = {"n_f": [], "m_f": [], "m_u": []}
    for d in range(L):
        in_f = (lv == d).any(axis=0)
        out["n_f"].append(int(in_f.sum()))
        out["m_f"].append(int(deg[in_f].sum()))
        out["m_u"].append(int(deg[done_at > d].sum()))
    return {k: np.array(v, dtype=np.int64) for k, v in out.items()}
