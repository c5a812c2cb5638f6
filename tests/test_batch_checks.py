"""CPU pins of the expected per-layer counters of a batched traversal
(tests/checks.batch_union_replay), which the GPU tests compare the batched
kernels' layer records with."""
from __future__ import annotations

import numpy as np

import inputs
import oracle
from tests import checks


def test_single_root_union_equals_layer_replay():
    g = inputs.kronecker(10)
    for r in inputs.pick_roots(g, 4, 3):
        lv, _ = oracle.bfs(g, int(r))
        rep = oracle.layer_replay(g, lv)
        u = checks.batch_union_replay(g, [lv])
        for k in ("n_f", "m_f", "m_u"):
            assert u[k].tolist() == rep[k].tolist(), k


def test_repeated_root_union_equals_single():
    g = inputs.grid_graph(9, 7)
    lv, _ = oracle.bfs(g, 20)
    one = checks.batch_union_replay(g, [lv])
    three = checks.batch_union_replay(g, [lv, lv, lv])
    for k in one:
        assert one[k].tolist() == three[k].tolist()


def test_two_ends_of_a_path_by_hand():
    """Path 0-1-2-3-4 from roots 0 and 4: F_0 = {0, 4}, F_1 = {1, 3}, F_2 = {2},
    F_3 = {1, 3}, F_4 = {0, 4}.  A vertex leaves m_u once both roots have
    reached it: 2 after layer 2, 1 and 3 after layer 3, 0 and 4 after layer 4."""
    g = inputs.path_graph(5)
    a, _ = oracle.bfs(g, 0)
    b, _ = oracle.bfs(g, 4)
    u = checks.batch_union_replay(g, [a, b])
    assert u["n_f"].tolist() == [2, 2, 1, 2, 2]
    assert u["m_f"].tolist() == [2, 4, 2, 4, 2]
    assert u["m_u"].tolist() == [8, 8, 6, 2, 0]


def test_unreachable_vertices_stay_in_m_u():
    g = inputs.from_edges(6, [(0, 1), (1, 2), (3, 4), (4, 5)])
    a, _ = oracle.bfs(g, 0)
    b, _ = oracle.bfs(g, 5)
    u = checks.batch_union_replay(g, [a, b])
    assert u["m_u"].tolist() == [8, 8, 8]
    assert u["n_f"].tolist() == [2, 2, 2]


def test_noncanonical_checker_accepts_valid_and_rejects_invalid_trees():
    """The first-writer validator (check_bfs_invariants(canonical=False)):
    a grid's tree with the largest closer neighbour as parent is accepted;
    a parent that is not adjacent, or one at the wrong level, is rejected."""
    import pytest
    g = inputs.grid_graph(6, 5)
    r = 7
    lv, pa = oracle.bfs(g, r)
    alt = pa.copy()
    for v in range(g.n):
        if lv[v] > 0:
            row = g.col[g.off[v]:g.off[v + 1]]
            alt[v] = max(u for u in row if lv[u] == lv[v] - 1)
    assert not np.array_equal(alt, pa)
    checks.check_bfs_invariants(g, r, lv, alt, canonical=False)
    with pytest.raises(AssertionError):
        checks.check_bfs_invariants(g, r, lv, alt)          # not canonical
    bad = alt.copy()
    far = int(np.argmax(lv))
    bad[far] = r                                            # not adjacent
    with pytest.raises(AssertionError):
        checks.check_bfs_invariants(g, r, lv, bad, canonical=False)
    bad = alt.copy()
    v = int(np.nonzero(lv == 2)[0][0])
    row = g.col[g.off[v]:g.off[v + 1]]
    bad[v] = int(next(u for u in row if lv[u] == 3))        # adjacent, one layer further
    with pytest.raises(AssertionError):
        checks.check_bfs_invariants(g, r, lv, bad, canonical=False)
