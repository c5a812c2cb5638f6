"""Batched multi-source BFS (bfs_run_batch) on the GPU: every root's level and
canonical parent arrays byte for byte equal to the oracle's single-root BFS,
for batch sizes around the 64-lane group boundary, repeated and isolated
roots, forced directions, tuning parameters, and edge-case graphs; the
per-layer union counters and the direction trace against the oracle's levels."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import inputs
import oracle
from tests import checks

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


@pytest.fixture(scope="module")
def hyb():
    import paper_1704_02259_amd as h
    h.load()
    return h


@pytest.fixture(scope="module")
def kron16(hyb):
    g = inputs.kronecker(16)
    return g, hyb.Graph.from_csr(g)


_expected_cache: dict = {}


def _expected(g, key, r):
    k = (key, int(r))
    if k not in _expected_cache:
        _expected_cache[k] = oracle.bfs(g, int(r))
    return _expected_cache[k]


def _gpu_batch(torch, G, roots, **kw):
    k = len(roots)
    lv = torch.empty(k * G.n, dtype=torch.int32, device="cuda")
    pa = torch.empty(k * G.n, dtype=torch.int32, device="cuda")
    out = G.run_batch(roots, lv, pa, stats=True, **kw)
    torch.cuda.synchronize()
    return lv.cpu().numpy().reshape(k, G.n), pa.cpu().numpy().reshape(k, G.n), out[2]


def _check_rows(g, key, roots, lv, pa):
    for i, r in enumerate(roots):
        elv, epa = _expected(g, key, r)
        bad = np.nonzero(lv[i] != elv)[0]
        assert len(bad) == 0, f"root #{i} ({r}): level mismatch at {bad[:8]} gpu={lv[i][bad[:8]]} " \
                              f"cpu={elv[bad[:8]]}"
        bad = np.nonzero(pa[i] != epa)[0]
        assert len(bad) == 0, f"root #{i} ({r}): parent mismatch at {bad[:8]} gpu={pa[i][bad[:8]]} " \
                              f"cpu={epa[bad[:8]]}"


def _check_stats(g, key, roots, st, rule="edges", alpha=14, beta=24):
    exp = [_expected(g, key, r)[0] for r in roots]
    assert st["reached"] == sum(int((e >= 0).sum()) for e in exp)
    assert st["reached_degree_sum"] == sum(oracle.reached_degree_sum(g, e) for e in exp)
    assert st["num_layers"] == max(int(e.max()) + 1 for e in exp)
    first = exp[:64]
    rep = checks.batch_union_replay(g, first)
    lay = st["layers"]
    L = len(rep["n_f"])
    assert len(lay) == L
    assert [x["n_f"] for x in lay] == rep["n_f"].tolist()
    assert [x["m_f"] for x in lay] == rep["m_f"].tolist()
    assert [x["m_u"] for x in lay] == rep["m_u"].tolist()
    orule = {"edges": "beamer", "td": "td", "bu": "bu"}[rule]
    rep = dict(rep, v_u=np.zeros(L, dtype=np.int64))
    assert [x["dir"] for x in lay] == oracle.direction_trace(orule, g.n, rep, alpha, beta).tolist()


def _kron16_roots(g, k, seed):
    """k roots: mostly degree > 0, with a repeated root and an isolated vertex."""
    rng = np.random.default_rng(seed)
    deg = np.diff(g.off)
    live = np.nonzero(deg > 0)[0]
    iso = np.nonzero(deg == 0)[0]
    r = rng.choice(live, size=k, replace=True).astype(np.int32)
    if k >= 3:
        r[1] = r[0]
        r[k // 2] = iso[0]
    return r


@pytest.mark.parametrize("k", [1, 2, 7, 63, 64, 65, 130])
def test_kron16_batch_sizes(torch, kron16, k):
    g, G = kron16
    roots = _kron16_roots(g, k, 100 + k)
    _say("kron16 batch k", k)
    lv, pa, st = _gpu_batch(torch, G, roots)
    _check_rows(g, "kron16", roots, lv, pa)
    _check_stats(g, "kron16", roots, st)


@pytest.mark.parametrize("rule", ["edges", "td", "bu"])
def test_kron16_batch_rules(torch, kron16, rule):
    g, G = kron16
    roots = _kron16_roots(g, 64, 7)
    _say("kron16 batch rule", rule)
    lv, pa, st = _gpu_batch(torch, G, roots, rule=rule)
    _check_rows(g, "kron16", roots, lv, pa)
    _check_stats(g, "kron16", roots, st, rule)


@pytest.mark.parametrize("grid,wpw,layers", [(1, 0, 0), (7, 1, 1), (0, 64, 3), (256, 2, 64), (0, 0, 1)])
def test_kron16_batch_parameters(torch, kron16, grid, wpw, layers):
    g, G = kron16
    roots = _kron16_roots(g, 40, 11)
    _say("kron16 batch params", grid, wpw, layers)
    lv, pa, st = _gpu_batch(torch, G, roots, grid_blocks=grid, words_per_wave=wpw, layers_per_launch=layers)
    _check_rows(g, "kron16", roots, lv, pa)


def test_kron16_batch_alpha_beta(torch, kron16):
    g, G = kron16
    roots = _kron16_roots(g, 64, 5)
    for a, b in ((1, 1), (2, 200), (100, 3), (10000, 10000)):
        _say("kron16 batch alpha beta", a, b)
        lv, pa, st = _gpu_batch(torch, G, roots, alpha=a, beta=b)
        _check_rows(g, "kron16", roots, lv, pa)
        _check_stats(g, "kron16", roots, st, "edges", a, b)


def test_batch_equals_single_runs(torch, kron16):
    """The batch is k independent traversals: equal to bfs_run per root."""
    g, G = kron16
    roots = _kron16_roots(g, 64, 9)
    lv, pa, _ = _gpu_batch(torch, G, roots)
    l1 = torch.empty(g.n, dtype=torch.int32, device="cuda")
    p1 = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for i, r in enumerate(roots):
        G.run(int(r), l1, p1)
        torch.cuda.synchronize()
        assert np.array_equal(l1.cpu().numpy(), lv[i]) and np.array_equal(p1.cpu().numpy(), pa[i]), i


def test_batch_host_outputs(torch, kron16):
    g, G = kron16
    roots = _kron16_roots(g, 70, 13)
    lv, pa = G.run_batch(roots)
    assert lv.shape == (70, g.n)
    _check_rows(g, "kron16", roots, lv, pa)


def test_batch_async_back_to_back(torch, kron16):
    g, G = kron16
    s = torch.cuda.Stream()
    sets = [_kron16_roots(g, 64, 21), _kron16_roots(g, 17, 22), _kron16_roots(g, 64, 23)]
    bufs = []
    for roots in sets:
        lv = torch.empty(len(roots) * g.n, dtype=torch.int32, device="cuda")
        pa = torch.empty(len(roots) * g.n, dtype=torch.int32, device="cuda")
        G.run_batch(roots, lv, pa, stream=s.cuda_stream, async_=1)
        bufs.append((lv, pa))
    s.synchronize()
    for roots, (lv, pa) in zip(sets, bufs):
        _check_rows(g, "kron16", roots, lv.cpu().numpy().reshape(-1, g.n), pa.cpu().numpy().reshape(-1, g.n))


def test_batch_graph_replay(torch, hyb, kron16):
    """graph_launch=1: each group of up to 64 roots is one hipGraph launch,
    captured once per group size and option set.  Replays with other roots,
    group sizes (17, 64, 130 = three groups), output buffers and layer counts,
    synchronous with stats, and asynchronous series on one stream (each replay
    rewrites the init and seed nodes while the previous one may still run),
    with direct runs and torch work between them; every replay against the
    oracle."""
    g, G = kron16
    sets = [_kron16_roots(g, 64, 41), _kron16_roots(g, 64, 42), _kron16_roots(g, 17, 43),
            _kron16_roots(g, 130, 44), _kron16_roots(g, 64, 45)]
    for roots in sets:
        _say("batch replay", len(roots), int(roots[0]))
        lv, pa, st = _gpu_batch(torch, G, roots, graph_launch=1)
        _check_rows(g, "kron16", roots, lv, pa)
        _check_stats(g, "kron16", roots, st)
        lv, pa, _ = _gpu_batch(torch, G, roots)          # a direct run between replays
        _check_rows(g, "kron16", roots, lv, pa)
    for roots in sets[:2]:
        lv, pa, st = _gpu_batch(torch, G, roots, graph_launch=1, layers_per_launch=2)
        _check_rows(g, "kron16", roots, lv, pa)
        _check_stats(g, "kron16", roots, st)
    s = torch.cuda.Stream()
    bufs = []
    for roots in sets + sets[::-1]:
        lv = torch.empty(len(roots) * g.n, dtype=torch.int32, device="cuda")
        pa = torch.empty(len(roots) * g.n, dtype=torch.int32, device="cuda")
        G.run_batch(roots, lv, pa, stream=s.cuda_stream, async_=1, graph_launch=1)
        bufs.append((roots, lv, pa))
    s.synchronize()
    for roots, lv, pa in bufs:
        _check_rows(g, "kron16", roots, lv.cpu().numpy().reshape(-1, g.n), pa.cpu().numpy().reshape(-1, g.n))
    for name, gs, roots in _small_cases():
        roots = np.array(roots, dtype=np.int32)
        Gs = hyb.Graph.from_csr(gs)
        for rep in range(2):
            lv, pa, st = _gpu_batch(torch, Gs, roots, graph_launch=1)
            _check_rows(gs, name, roots, lv, pa)
            _check_stats(gs, name, roots, st)
        Gs.close()


def _small_cases():
    yield "path1000", inputs.path_graph(1000), [0, 500, 999, 0, 1]
    yield "cycle257", inputs.cycle_graph(257), [0, 128, 256]
    yield "grid33x17", inputs.grid_graph(33, 17), [0, 33 * 17 // 2, 33 * 17 - 1]
    yield "star300c", inputs.star_graph(300, center=150), [150, 3, 299, 150]
    yield "K65", inputs.complete_graph(65), list(range(65))[:64]
    yield "Q9", inputs.hypercube_graph(9), [0, 311, 511]
    yield "gnp200", inputs.random_graph(200, 0.01, 3), list(range(0, 200, 3))[:64]
    yield "n1", inputs.from_edges(1, []), [0]
    yield "edgeless5", inputs.from_edges(5, []), [3, 0, 4]
    yield "n63", inputs.random_graph(63, 0.1, 8), [0, 62]
    yield "n65", inputs.random_graph(65, 0.1, 9), [64, 0]
    yield "isolated_root", inputs.from_edges(130, [(0, 1), (1, 2), (100, 129)]), [50, 129, 0, 2]


@pytest.mark.parametrize("case", list(_small_cases()), ids=lambda c: c[0])
def test_batch_edge_case_graphs(torch, hyb, case):
    name, g, roots = case
    roots = np.array(roots, dtype=np.int32)
    G = hyb.Graph.from_csr(g)
    for rule in ("edges", "td", "bu"):
        _say(name, rule, len(roots))
        lv, pa, st = _gpu_batch(torch, G, roots, rule=rule)
        _check_rows(g, name, roots, lv, pa)
        _check_stats(g, name, roots, st, rule)
    G.close()


def _kept_layers():
    """kBatchHist, the layers whose frontier masks a batch keeps, as the
    kernels' header defines it."""
    import os
    import re
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with open(os.path.join(root, "paper_1704_02259_amd", "csrc", "bfs_device.h")) as f:
        m = re.search(r"constexpr int kBatchHist = (\d+);", f.read())
    assert m, "kBatchHist not found"
    return int(m.group(1))


def test_batch_depths_around_kept_layers(torch, hyb):
    """The levels of a batch's first layers are stored after the traversal
    from the kept frontier masks, the deeper ones by their layers (and the
    finisher): paths whose depths end just below, at and above that boundary,
    with lanes of different depths in one batch, several launch depths, graph
    replays, and deep and shallow batches in turn on one workspace (the kept
    masks must be clear again for the next batch)."""
    H = _kept_layers()
    for n in (H - 1, H, H + 1, H + 2, 3 * H + 5):
        g = inputs.path_graph(n)
        G = hyb.Graph.from_csr(g)
        sets = [[0], [n - 1, 0, n // 2], [n // 2], [0, n - 1] * 3, [n // 3, 1]]
        for i, roots in enumerate(sets):
            roots = np.array(roots, dtype=np.int32)
            for kw in ({}, {"layers_per_launch": 1}, {"layers_per_launch": H}, {"layers_per_launch": H + 1},
                       {"graph_launch": 1}, {"graph_launch": 1, "layers_per_launch": 2}):
                _say("path", n, "set", i, kw)
                lv, pa, st = _gpu_batch(torch, G, roots, **kw)
                _check_rows(g, f"path{n}", roots, lv, pa)
                _check_stats(g, f"path{n}", roots, st)
        G.close()


def test_batch_after_a_failed_batch(torch, hyb):
    """A batch that fails a device-side check (forced from the host with the
    library's test hook: the finisher reports the traversal as failed while
    every kernel runs normally) is reported, and the next batches on the same
    workspace are exact: the level pass clears every kept mask after a
    failure."""
    import os
    from paper_1704_02259_amd import hybfs
    g = inputs.kronecker(12)
    roots = [int(r) for r in inputs.pick_roots(g, 5, 2212)]
    old = os.environ.pop("HYBFS_TEST_FAIL_ROOT", None)
    try:
        os.environ["HYBFS_TEST_FAIL_ROOT"] = str(roots[0])
        G = hyb.Graph.from_csr(g)
    finally:
        os.environ.pop("HYBFS_TEST_FAIL_ROOT", None)
        if old is not None:
            os.environ["HYBFS_TEST_FAIL_ROOT"] = old
    for kw in ({}, {"graph_launch": 1}):
        _say("failing batch", kw)
        with pytest.raises(hybfs.HybfsError) as ei:
            _gpu_batch(torch, G, np.array(roots, dtype=np.int32), **kw)
        assert ei.value.code == hybfs.BFS_E_DEVICE
        for sub in (roots[1:], roots[2:4]):
            sub = np.array(sub, dtype=np.int32)
            _say("batch after the failure", kw, list(sub))
            lv, pa, st = _gpu_batch(torch, G, sub, **kw)
            _check_rows(g, "kron12", sub, lv, pa)
            _check_stats(g, "kron12", sub, st)
    G.close()


def test_batch_unsorted_rows(torch, hyb):
    base = inputs.kronecker(10)
    rng = np.random.default_rng(4)
    dirty = inputs.CSR(base.n, base.off.copy(), base.col.copy())
    for v in range(dirty.n):
        rng.shuffle(dirty.col[dirty.off[v]:dirty.off[v + 1]])
    from paper_1704_02259_amd import hybfs
    G = hyb.Graph.from_csr(dirty, flags=hybfs.BFS_GRAPH_SORT_ROWS)
    roots = inputs.pick_roots(base, 64, 5).astype(np.int32)
    lv, pa, _ = _gpu_batch(torch, G, roots)
    _check_rows(base, "kron10", roots, lv, pa)
    G.close()


def test_batch_invalid_arguments(torch, kron16):
    from paper_1704_02259_amd import hybfs
    g, G = kron16
    for roots, kw in (([0, g.n], {}), ([-1], {}), ([0], {"rule": "table"})):
        with pytest.raises(hybfs.HybfsError) as ei:
            G.run_batch(roots, **kw)
        assert ei.value.code == hybfs.BFS_E_INVALID
    with pytest.raises(hybfs.HybfsError):
        G.run_batch([])


# ---------------------------------------------------------------- SCALE 20
@pytest.fixture(scope="module")
def kron20(hyb):
    g = inputs.kronecker(20)
    return g, hyb.Graph.from_csr(g), inputs.workload_roots("kron20", g, 64)


def test_kron20_batch_64_roots(torch, kron20):
    """The 64 roots of the SCALE-20 workload in one group: four rows against
    the oracle, every row against the O(nnz) invariants, and the totals."""
    g, G, roots = kron20
    roots = np.asarray(roots, dtype=np.int32)
    lv, pa, st = _gpu_batch(torch, G, roots)
    _check_rows(g, "kron20", roots[:4], lv[:4], pa[:4])
    tot = 0
    for i, r in enumerate(roots):
        checks.check_bfs_invariants(g, int(r), lv[i], pa[i], None)
        tot += oracle.reached_degree_sum(g, lv[i])
    assert st["reached_degree_sum"] == tot


def test_autotune_batch_keeps_results(torch, kron16):
    g, G = kron16
    opts, rep = G.autotune(_kron16_roots(g, 64, 31), mode="batch", max_trials=10)
    _say("autotune batch", opts, rep)
    assert 1 <= rep["trials"] <= 10
    roots = _kron16_roots(g, 64, 32)
    kw = {k: v for k, v in opts.items() if k != "probe_k"}
    lv, pa, st = _gpu_batch(torch, G, roots, **kw)
    _check_rows(g, "kron16", roots, lv, pa)
