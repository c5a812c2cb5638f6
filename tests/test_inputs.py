"""Structure and determinism of the seeded input graphs."""
import numpy as np
import pytest

import inputs


def _structure_ok(g):
    off, col = g.off, g.col
    assert off[0] == 0 and np.all(np.diff(off) >= 0) and off[-1] == len(col)
    assert col.dtype == np.int32 and off.dtype == np.int64
    assert np.all((col >= 0) & (col < g.n))
    src = np.repeat(np.arange(g.n), np.diff(off))
    assert not np.any(src == col), "self-loop"
    # rows strictly ascending -> sorted and duplicate free
    same_row = src[1:] == src[:-1]
    assert np.all(col[1:][same_row] > col[:-1][same_row])
    # symmetric
    key = src.astype(np.int64) * g.n + col
    rkey = col.astype(np.int64) * g.n + src
    assert np.array_equal(np.sort(key), np.sort(rkey))
    assert g.nnz % 2 == 0


@pytest.mark.parametrize("scale", [4, 8, 12, 16])
def test_kronecker_structure(scale):
    _structure_ok(inputs.kronecker(scale))


def test_kronecker_deterministic_and_seeded():
    a, b = inputs.kronecker(12), inputs.kronecker(12)
    c = inputs.kronecker(12, seed=99)
    assert np.array_equal(a.off, b.off) and np.array_equal(a.col, b.col)
    assert not np.array_equal(a.col[:1000], c.col[:1000])


def test_kronecker_distribution():
    # Power-law structure of the A/B/C/D initiator at SCALE 16, edgefactor 16:
    # about 29% isolated vertices and nnz ~ 0.87 of the 2*16*2^16 directed draws.
    g = inputs.kronecker(16)
    deg = g.degrees()
    assert 0.25 < (deg == 0).mean() < 0.33
    assert 0.84 < g.nnz / (2 * 16 * g.n) < 0.90
    assert deg.max() > 3000


def test_erdos_renyi_structure():
    g = inputs.erdos_renyi(1 << 14, 4 << 14, seed=5)
    _structure_ok(g)
    assert abs(g.nnz / g.n - 8.0) < 0.1


def test_roots_distinct_nonzero_degree():
    g = inputs.kronecker(12)
    r = inputs.pick_roots(g, 64, 2012)
    assert len(np.unique(r)) == 64
    assert np.all(g.degrees()[r] > 0)
    assert np.array_equal(r, inputs.pick_roots(g, 64, 2012))


def test_small_families():
    for g in (inputs.path_graph(7), inputs.cycle_graph(9), inputs.grid_graph(3, 4),
              inputs.star_graph(6), inputs.complete_graph(5), inputs.hypercube_graph(3),
              inputs.random_graph(30, 0.1, 1)):
        _structure_ok(g)
