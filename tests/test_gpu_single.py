"""Single-root hybrid BFS on the GPU against the CPU oracle: levels and
canonical parents byte for byte, per-layer counters and direction trace equal
to the oracle's replay, on Kronecker graphs (SCALE 16 with 4 roots, sampled
roots at SCALE 20) and on edge-case graphs."""
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


def _gpu_bfs(torch, G, root, **kw):
    lv = torch.empty(G.n, dtype=torch.int32, device="cuda")
    pa = torch.empty(G.n, dtype=torch.int32, device="cuda")
    out = G.run(root, lv, pa, stats=True, **kw)
    torch.cuda.synchronize()
    return lv.cpu().numpy(), pa.cpu().numpy(), out[2]


def _check_against_oracle(g, root, lv, pa, st=None, rule="edges", alpha=14, beta=24):
    elv, epa = oracle.bfs(g, root)
    bad = np.nonzero(lv != elv)[0]
    assert len(bad) == 0, f"level mismatch at {bad[:8]} gpu={lv[bad[:8]]} cpu={elv[bad[:8]]}"
    bad = np.nonzero(pa != epa)[0]
    assert len(bad) == 0, f"parent mismatch at {bad[:8]} gpu={pa[bad[:8]]} cpu={epa[bad[:8]]}"
    if st is not None:
        rep = oracle.layer_replay(g, elv)
        L = len(rep["n_f"])
        assert st["num_layers"] == L
        lay = st["layers"]
        assert [x["n_f"] for x in lay] == rep["n_f"].tolist()
        assert [x["m_f"] for x in lay] == rep["m_f"].tolist()
        assert [x["m_u"] for x in lay] == rep["m_u"].tolist()
        assert [x["v_u"] for x in lay] == rep["v_u"].tolist()
        orule = {"edges": "beamer", "table": "table", "td": "td", "bu": "bu"}[rule]
        exp_dir = oracle.direction_trace(orule, g.n, rep, alpha, beta)
        assert [x["dir"] for x in lay] == exp_dir.tolist()
        assert st["reached"] == int((elv >= 0).sum())
        assert st["reached_degree_sum"] == oracle.reached_degree_sum(g, elv)


@pytest.fixture(scope="module")
def kron16(hyb):
    g = inputs.kronecker(16)
    return g, hyb.Graph.from_csr(g), inputs.workload_roots("kron16", g, 4)


@pytest.mark.parametrize("rule", ["edges", "td", "bu", "table"])
def test_kron16_four_roots(torch, kron16, rule):
    g, G, roots = kron16
    for r in roots:
        _say("kron16 rule", rule, "root", int(r))
        lv, pa, st = _gpu_bfs(torch, G, int(r), rule=rule)
        _check_against_oracle(g, int(r), lv, pa, st, rule)


@pytest.mark.parametrize("probe_k,hubdeg,grid,wpw,layers",
                         [(0, 256, 0, 0, 0), (1, 4096, 1, 1, 1), (3, 257, 7, 64, 3),
                          (8, 1 << 24, 0, 2, 40), (64, 512, 33, 16, 2)])
def test_kron16_parameters_do_not_change_output(torch, kron16, probe_k, hubdeg, grid, wpw, layers):
    g, G, roots = kron16
    r = int(roots[0])
    kw = dict(probe_k=probe_k, td_hub_degree=hubdeg, grid_blocks=grid, words_per_wave=wpw,
              bu_serial_probes=1 if probe_k % 2 else -1,
              layers_per_launch=layers, graph_launch=layers % 2)
    _say("kron16 params", kw)
    lv, pa, st = _gpu_bfs(torch, G, r, **kw)
    _check_against_oracle(g, r, lv, pa, st)
    lv2, pa2, _ = _gpu_bfs(torch, G, r, rule="bu", **kw)
    assert np.array_equal(lv, lv2) and np.array_equal(pa, pa2)
    lv3, pa3, _ = _gpu_bfs(torch, G, r, rule="td", **kw)
    assert np.array_equal(lv, lv3) and np.array_equal(pa, pa3)


def test_kron16_alpha_beta_sweep(torch, kron16):
    g, G, roots = kron16
    r = int(roots[1])
    for a, b in [(1, 1), (2, 100), (14, 24), (1000, 2), (100000, 100000)]:
        _say("kron16 alpha/beta", a, b)
        lv, pa, st = _gpu_bfs(torch, G, r, alpha=a, beta=b)
        _check_against_oracle(g, r, lv, pa, st, "edges", a, b)


def test_repeat_runs_are_identical(torch, kron16):
    g, G, roots = kron16
    r = int(roots[2])
    a = _gpu_bfs(torch, G, r)
    for _ in range(5):
        b = _gpu_bfs(torch, G, r)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_host_outputs_equal_device_outputs(torch, hyb, kron16):
    g, G, roots = kron16
    r = int(roots[3])
    lv, pa = G.run(r)              # numpy (host) outputs, pageable memory
    lv2, pa2, _ = _gpu_bfs(torch, G, r)
    assert np.array_equal(lv, lv2) and np.array_equal(pa, pa2)
    _check_against_oracle(g, r, lv, pa)
    # pinned host buffers, filled with garbage first, on an explicit stream
    lvp = torch.full((g.n,), 7, dtype=torch.int32, pin_memory=True)
    pap = torch.full((g.n,), 7, dtype=torch.int32, pin_memory=True)
    s = torch.cuda.Stream()
    opt = hyb.hybfs.bfs_options_init(out_on_device=0, stream=s.cuda_stream)
    hyb.hybfs.bfs_run(G.handle, r, lvp.data_ptr(), pap.data_ptr(), opt, None)
    assert np.array_equal(lvp.numpy(), lv2) and np.array_equal(pap.numpy(), pa2)


def _small_cases():
    yield "path1000", inputs.path_graph(1000), [0, 500, 999]
    yield "path70", inputs.path_graph(70), [0, 69]
    yield "cycle257", inputs.cycle_graph(257), [0, 128]
    yield "grid33x17", inputs.grid_graph(33, 17), [0, 33 * 17 // 2, 33 * 17 - 1]
    yield "star300c", inputs.star_graph(300, center=150), [150, 3, 299]
    yield "K65", inputs.complete_graph(65), [0, 64]
    yield "Q9", inputs.hypercube_graph(9), [0, 311]
    yield "gnp200", inputs.random_graph(200, 0.01, 3), [0, 1, 77]
    yield "n1", inputs.from_edges(1, []), [0]
    yield "edgeless5", inputs.from_edges(5, []), [3]
    yield "n63", inputs.random_graph(63, 0.1, 8), [0, 62]
    yield "n65", inputs.random_graph(65, 0.1, 9), [64]
    yield "isolated_root", inputs.from_edges(130, [(0, 1), (1, 2), (100, 129)]), [50, 129]


@pytest.mark.parametrize("case", list(_small_cases()), ids=lambda c: c[0])
def test_edge_case_graphs(torch, hyb, case):
    name, g, roots = case
    G = hyb.Graph.from_csr(g)
    for rule in ("edges", "td", "bu", "table"):
        for r in roots:
            _say(name, rule, r)
            lv, pa, st = _gpu_bfs(torch, G, r, rule=rule)
            _check_against_oracle(g, r, lv, pa, st, rule)
    G.close()


@pytest.mark.parametrize("case", list(_small_cases()), ids=lambda c: c[0])
def test_edge_case_graphs_binned_top_down(torch, hyb, case):
    """Every top-down layer through the binned path (td_binned=1): buckets
    per destination tile, minima in LDS, tile-wise outputs."""
    name, g, roots = case
    G = hyb.Graph.from_csr(g)
    for rule in ("edges", "td"):
        for r in roots:
            _say(name, "binned", rule, r)
            lv, pa, st = _gpu_bfs(torch, G, r, rule=rule, td_binned=1)
            _check_against_oracle(g, r, lv, pa, st, rule)
    G.close()


def test_unsorted_rows_duplicates_and_self_loops(torch, hyb):
    base = inputs.kronecker(10)
    rng = np.random.default_rng(1)
    src = np.repeat(np.arange(base.n), np.diff(base.off))
    edges = np.stack([src, base.col], 1)
    extra = np.stack([np.arange(0, base.n, 7), np.arange(0, base.n, 7)], 1)  # self-loops
    dup = edges[rng.integers(0, len(edges), 500)]
    dirty = inputs.from_edges(base.n, np.concatenate([edges, extra, dup]), keep_self_loops=True,
                              keep_duplicates=True, sort_rows=False)
    for v in range(dirty.n):
        rng.shuffle(dirty.col[dirty.off[v]:dirty.off[v + 1]])
    from paper_1704_02259_amd import hybfs
    G = hyb.Graph.from_csr(dirty, flags=hybfs.BFS_GRAPH_SORT_ROWS)
    for r in inputs.pick_roots(base, 3, 4):
        lv, pa, st = _gpu_bfs(torch, G, int(r))
        _check_against_oracle(base, int(r), lv, pa)
    G.close()


@pytest.mark.parametrize("rule", ["edges", "td"])
def test_kron16_binned_top_down(torch, kron16, rule):
    g, G, roots = kron16
    for r in roots:
        _say("kron16 binned", rule, int(r))
        lv, pa, st = _gpu_bfs(torch, G, int(r), rule=rule, td_binned=1)
        _check_against_oracle(g, int(r), lv, pa, st, rule)
    # and with the hub cut-off raised, the grid shrunk, several task sizes
    for kw in (dict(td_hub_degree=4096), dict(grid_blocks=3, words_per_wave=1), dict(td_hub_degree=1024,
                                                                                     words_per_wave=8),
               dict(bu_serial_probes=1), dict(bu_serial_probes=1, probe_k=16)):
        lv, pa, st = _gpu_bfs(torch, G, int(roots[0]), rule=rule, td_binned=1, **kw)
        _check_against_oracle(g, int(roots[0]), lv, pa, st, rule)


def test_kron18_binned_many_tiles(torch, hyb):
    """SCALE 18: eight destination tiles; binned on every top-down layer and
    off entirely give the oracle's result."""
    g = inputs.kronecker(18)
    G = hyb.Graph.from_csr(g)
    for r in inputs.workload_roots("kron18", g, 3):
        for tb in (1, -1):
            _say("kron18 binned", tb, int(r))
            lv, pa, st = _gpu_bfs(torch, G, int(r), td_binned=tb)
            _check_against_oracle(g, int(r), lv, pa, st)
        lv, pa, st = _gpu_bfs(torch, G, int(r), rule="td", td_binned=1)
        _check_against_oracle(g, int(r), lv, pa, st, "td")
    G.close()


def test_invalid_root_is_rejected(torch, kron16):
    from paper_1704_02259_amd import hybfs
    g, G, _ = kron16
    with pytest.raises(hybfs.HybfsError) as ei:
        G.run(g.n)
    assert ei.value.code == hybfs.BFS_E_INVALID


def test_two_streams_concurrently(torch, kron16):
    import threading
    g, G, roots = kron16
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    res = {}

    def work(key, stream, r):
        lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
        pa = torch.empty(g.n, dtype=torch.int32, device="cuda")
        for _ in range(3):
            G.run(r, lv, pa, stream=stream.cuda_stream)
        stream.synchronize()
        res[key] = (lv.cpu().numpy(), pa.cpu().numpy())

    t1 = threading.Thread(target=work, args=("a", s1, int(roots[0])))
    t2 = threading.Thread(target=work, args=("b", s2, int(roots[1])))
    t1.start(); t2.start(); t1.join(); t2.join()
    for key, r in (("a", roots[0]), ("b", roots[1])):
        _check_against_oracle(g, int(r), *res[key])


# ---------------------------------------------------------------- SCALE 20
@pytest.fixture(scope="module")
def kron20(hyb):
    g = inputs.kronecker(20)
    return g, hyb.Graph.from_csr(g), inputs.workload_roots("kron20", g, 64)


def test_kron20_sampled_roots_exact(torch, kron20):
    g, G, roots = kron20
    comp = None
    for r in roots[:4]:
        _say("kron20 root", int(r))
        lv, pa, st = _gpu_bfs(torch, G, int(r))
        _check_against_oracle(g, int(r), lv, pa, st)


def test_kron20_binned_top_down(torch, kron20):
    g, G, roots = kron20
    for r in roots[:3]:
        _say("kron20 binned", int(r))
        lv, pa, st = _gpu_bfs(torch, G, int(r), td_binned=1)
        _check_against_oracle(g, int(r), lv, pa, st)


def test_kron20_all_roots_invariants(torch, kron20):
    """All 64 roots of the SCALE-20 workload: O(nnz) invariant checks per root
    (tree edges, layer spans, canonical parent as the minimum closer
    neighbour), plus the reached set against one union-find labelling."""
    g, G, roots = kron20
    comp = checks.components(g) if g.n <= (1 << 16) else None
    lv0 = None
    for r in roots:
        lv, pa, st = _gpu_bfs(torch, G, int(r))
        checks.check_bfs_invariants(g, int(r), lv, pa, comp)
        if lv0 is None:
            lv0 = lv
        # every root of degree > 0 in the giant component reaches the same set
        assert st["reached"] == int((lv >= 0).sum())


def test_graph_replay_alternating_roots_and_buffers(torch, kron16):
    """The captured launch sequence (graph_launch=1) is replayed with a new root
    and new output buffers each time; every replay must match the oracle, as
    must the direct (kernel-by-kernel) launch."""
    g, G, roots = kron16
    bufs = [(torch.empty(g.n, dtype=torch.int32, device="cuda"),
             torch.empty(g.n, dtype=torch.int32, device="cuda")) for _ in range(3)]
    expected = {int(r): oracle.bfs(g, int(r)) for r in roots}
    for it in range(9):
        r = int(roots[it % len(roots)])
        lv, pa = bufs[it % 3]
        G.run(r, lv, pa, graph_launch=1)
        torch.cuda.synchronize()
        assert np.array_equal(lv.cpu().numpy(), expected[r][0]), (it, r)
        assert np.array_equal(pa.cpu().numpy(), expected[r][1]), (it, r)
    for r in roots:
        lv, pa, st = _gpu_bfs(torch, G, int(r), graph_launch=0)
        _check_against_oracle(g, int(r), lv, pa, st)


def test_wide_layer_kernel_direct_and_graph_replay(torch, hyb):
    """From 2^24 vertices the layers run in the wide build of the layer kernel
    (more wavefronts per SIMD, six blocks per CU).  A sparse 2^24-vertex graph
    (Erdos-Renyi, mean degree 3, about 24 layers) traversed by direct launches
    and by hipGraph replays, both byte for byte against the oracle."""
    g = inputs.erdos_renyi(1 << 24, 3 << 23, seed=2424)
    G = hyb.Graph.from_csr(g)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert G.info().grid_blocks > 5 * cus      # the wide launch shape was chosen
    assert G.info().layer_kernel_wide == 1
    small = hyb.Graph.from_csr(inputs.path_graph(100))
    assert small.info().layer_kernel_wide == 0
    small.close()
    for r in inputs.pick_roots(g, 2, 77):
        r = int(r)
        _say("er2^24 root", r)
        exp = oracle.bfs(g, r)
        for graph in (0, 1, 1):
            lv, pa, st = _gpu_bfs(torch, G, r, graph_launch=graph)
            assert np.array_equal(lv, exp[0]) and np.array_equal(pa, exp[1]), (r, graph)
    G.close()


def test_async_runs_back_to_back(torch, kron16):
    """Asynchronous runs enqueued back to back on one stream, each into its own
    buffers, then one synchronisation."""
    g, G, roots = kron16
    s = torch.cuda.Stream()
    outs = []
    for r in list(roots) * 2:
        lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
        pa = torch.empty(g.n, dtype=torch.int32, device="cuda")
        G.run(int(r), lv, pa, stream=s.cuda_stream, async_=1)
        outs.append((int(r), lv, pa))
    from paper_1704_02259_amd import hybfs
    hybfs.bfs_graph_sync(G.handle, s.cuda_stream)
    for r, lv, pa in outs:
        elv, epa = oracle.bfs(g, r)
        assert np.array_equal(lv.cpu().numpy(), elv) and np.array_equal(pa.cpu().numpy(), epa)


def test_mixed_launch_paths_on_one_stream(torch, kron16):
    """One stream, one workspace: asynchronous runs that alternate the
    captured graph (plain initialisation, grid-wide layer 0), the fused
    initialisation with layer 0 (roots of degree <= 4096) and the grid-wide
    layer 0 of a high-degree root.  The fused kernel relies on the counters
    the previous traversal's finisher cleared, whichever path that traversal
    took; every output equals the oracle's."""
    g, G, roots = kron16
    deg = np.diff(g.off)
    hub = int(np.argmax(deg))
    seq = [(int(roots[0]), 1), (int(roots[1]), 0), (hub, 0), (int(roots[2]), 0), (int(roots[3]), 1),
           (int(roots[0]), 0), (hub, 1), (int(roots[1]), 0)]
    s = torch.cuda.Stream()
    outs = []
    for r, graph in seq:
        lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
        pa = torch.empty(g.n, dtype=torch.int32, device="cuda")
        G.run(r, lv, pa, stream=s.cuda_stream, async_=1, graph_launch=graph)
        outs.append((r, lv, pa))
    from paper_1704_02259_amd import hybfs
    hybfs.bfs_graph_sync(G.handle, s.cuda_stream)
    for r, lv, pa in outs:
        elv, epa = oracle.bfs(g, r)
        assert np.array_equal(lv.cpu().numpy(), elv) and np.array_equal(pa.cpu().numpy(), epa), r


def test_autotune_single_keeps_results(torch, kron16):
    """bfs_autotune (single-root mode) on other roots; the options it returns
    are valid and leave every root's output byte-identical to the oracle."""
    g, G, roots = kron16
    tune_roots = inputs.pick_roots(g, 8, 77)
    opts, rep = G.autotune(tune_roots, mode="single", max_trials=14)
    _say("autotune single", opts, rep)
    assert 1 <= rep["trials"] <= 14 and rep["best_us"] <= rep["start_us"] + 1e-9
    assert opts["td_hub_degree"] >= 256
    for r in roots:
        lv, pa, st = _gpu_bfs(torch, G, int(r), **opts)
        _check_against_oracle(g, int(r), lv, pa)


@pytest.mark.parametrize("rule", ["edges", "td"])
def test_first_writer_parents(torch, kron16, hyb, rule):
    """first_writer=1 (Algorithm 1's first-writer parents): levels and layer
    counters still equal the oracle's; parents are valid BFS-tree parents
    (a neighbour one layer closer), checked by the invariants."""
    g, G, roots = kron16
    for r in roots:
        lv, pa, st = _gpu_bfs(torch, G, int(r), rule=rule, first_writer=1)
        elv, _ = oracle.bfs(g, int(r))
        assert np.array_equal(lv, elv)
        checks.check_bfs_invariants(g, int(r), lv, pa, canonical=False)
        rep = oracle.layer_replay(g, elv)
        assert [x["n_f"] for x in st["layers"]] == rep["n_f"].tolist()
    for name, gg, rr in list(_small_cases())[:8]:
        GG = hyb.Graph.from_csr(gg)
        for r in rr:
            lv, pa, st = _gpu_bfs(torch, GG, r, rule="td", first_writer=1)
            assert np.array_equal(lv, oracle.bfs(gg, r)[0]), name
            checks.check_bfs_invariants(gg, r, lv, pa, canonical=False)
        GG.close()
    # the captured launch sequence keys on the parent mode
    lv, pa, _ = _gpu_bfs(torch, G, int(roots[0]), graph_launch=1, first_writer=1)
    checks.check_bfs_invariants(g, int(roots[0]), lv, pa, canonical=False)
    lv, pa, _ = _gpu_bfs(torch, G, int(roots[0]), graph_launch=1)
    _check_against_oracle(g, int(roots[0]), lv, pa)


def test_root_degree_paths(torch, kron16, hyb):
    """Layer 0 runs inside the initialisation kernel for roots of degree <=
    4096 and in the grid kernel above that: the highest-degree vertex, a
    degree-4096-ish vertex and a leaf, in an order that alternates the two
    paths on one workspace, all give the oracle's output and per-layer
    counters."""
    g, G, _ = kron16
    deg = np.diff(g.off)
    order = np.argsort(deg)
    picks = [int(order[-1]), int(order[np.searchsorted(deg[order], 4096, side="right") - 1]),
             int(order[np.searchsorted(deg[order], 1)]), int(order[-1])]
    for r in picks:
        _say("root degree", int(deg[r]))
        lv, pa, st = _gpu_bfs(torch, G, r)
        _check_against_oracle(g, r, lv, pa, st)
        assert st["layer0_kernel"] == (2 if deg[r] <= 4096 else 0)
        lv, pa, st = _gpu_bfs(torch, G, r, rule="bu")
        _check_against_oracle(g, r, lv, pa, st, "bu")


def test_root_kernel_when_ranges_exceed_lds(torch, hyb):
    """With a one-block grid on a graph of more than 2^16 vertices a block's
    share of the bitmap exceeds what the fused initialisation kernel stages in
    LDS, so layer 0 runs in its own one-block kernel; the default grid fuses
    it.  Both give the oracle's output, also back to back on one stream."""
    g = inputs.kronecker(17)
    G = hyb.Graph.from_csr(g)
    d = np.diff(g.off)
    roots = [int(v) for v in np.nonzero((d > 0) & (d <= 4096))[0][:3]]
    for grid in (1, 0, 1):
        for r in roots:
            _say("kron17 root", r, "grid", grid)
            lv, pa, st = _gpu_bfs(torch, G, r, grid_blocks=grid)
            _check_against_oracle(g, r, lv, pa, st)
            assert st["layer0_kernel"] == (1 if grid == 1 else 2)
    G.close()


def test_graph_replay_fused_init_and_binned_nodes(torch, kron16, hyb):
    """The captured launch sequence runs layer 0 in the initialisation node
    for roots of small degree (a second graph, with the grid-wide layer 0,
    for the others) and carries the binned top-down kernels when layers may
    bin: replays alternating the two graphs, with and without binning, async
    and sync, all equal to the oracle; layer0_kernel reports the form."""
    g, G, roots = kron16
    deg = np.diff(g.off)
    big = int(np.argmax(deg))
    lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
    pa = torch.empty(g.n, dtype=torch.int32, device="cuda")
    seq = [int(roots[0]), big, int(roots[1]), big, int(roots[2])]
    for tb in (0, 1, -1):
        for r in seq:
            G.run(r, lv, pa, async_=1, graph_launch=1, td_binned=tb)
        hyb.hybfs.bfs_graph_sync(G.handle, torch.cuda.current_stream().cuda_stream)
        for r in seq:
            _say("graph replay", r, "binned", tb)
            a = _gpu_bfs(torch, G, r, graph_launch=1, td_binned=tb)
            _check_against_oracle(g, r, a[0], a[1], a[2])
            assert a[2]["layer0_kernel"] == (2 if deg[r] <= 4096 else 0)


def test_library_first_then_torch():
    """A fresh process that loads the library and runs a traversal before it
    touches torch still finds torch's GPU afterwards, and both agree (torch's
    runtime starts first inside load())."""
    import subprocess
    code = (
        "import numpy as np, inputs, oracle\n"
        "from paper_1704_02259_amd import hybfs\n"
        "hybfs.load()\n"
        "g = inputs.kronecker(10)\n"
        "G = hybfs.Graph.from_csr(g)\n"
        "r = int(inputs.pick_roots(g, 1, 7)[0])\n"
        "lv, pa = G.run(r)[:2]\n"
        "import torch\n"
        "assert torch.cuda.is_available(), 'torch lost the GPU'\n"
        "l2 = torch.empty(g.n, dtype=torch.int32, device='cuda')\n"
        "p2 = torch.empty(g.n, dtype=torch.int32, device='cuda')\n"
        "G.run(r, l2, p2)\n"
        "torch.cuda.synchronize()\n"
        "elv, epa = oracle.bfs(g, r)\n"
        "assert np.array_equal(lv, elv) and np.array_equal(pa, epa)\n"
        "assert np.array_equal(l2.cpu().numpy(), elv) and np.array_equal(p2.cpu().numpy(), epa)\n"
        "print('ok')\n")
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=180)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok"), out.stdout[-2000:] + out.stderr[-2000:]


def test_autotune_table_round_trip(torch, hyb, tmp_path):
    """Tuning records its options in a table; a later call with the table
    returns them without tuning, and they leave the results unchanged."""
    g = inputs.kronecker(14)
    G = hyb.Graph.from_csr(g)
    roots = [int(r) for r in inputs.pick_roots(g, 8, 1414)]
    table = str(tmp_path / "tune.jsonl")
    o1, r1 = G.autotune(roots, max_trials=8, table=table, write_table=table)
    assert r1["source"] == "tuned" and r1["trials"] >= 1
    o2, r2 = G.autotune(roots, max_trials=8, table=table)
    assert r2["source"] == "table" and r2["trials"] == 0 and o2 == o1
    assert abs(r2["best_us"] - r1["best_us"]) < 1e-2
    ob, rb = G.autotune(roots, mode="batch", max_trials=4, table=table, write_table=table)
    assert rb["source"] == "tuned"                      # the batched mode has its own entry
    assert G.autotune(roots, mode="batch", table=table)[1]["source"] == "table"
    kw = {k: v for k, v in o2.items() if k not in ("rule",)}
    for r in roots[:3]:
        lv, pa, st = _gpu_bfs(torch, G, r, **kw)
        _check_against_oracle(g, r, lv, pa)
    G.close()
