"""Frontier queues and hub lists (options td_queue and td_hub_list) against the
CPU oracle: levels and canonical parents byte for byte and per-layer counters
equal to the oracle's replay, whatever mode writes and reads the queues:

  td_queue=1    top-down layers (and layer 0) append what they discover to
                the next frontier's queue; a top-down layer after them reads it
  td_queue=2    every layer writes its output as a queue too (the bottom-up
                and binned steps convert their output bitmap words), so every
                top-down layer reads a queue
  td_hub_list=1 the steps that discover vertices above the top-down cut-off
                list their edge chunks; top-down layers expand hubs from it
  td_hub_list=2 only layer 0 lists them, for layer 1
  td_hub_list=3 layer 0 and the top-down steps list them
  td_hub_list=4 layer 0 and a top-down layer 1 list them

Covered: every direction rule on edge-case graphs and Kronecker SCALE 16 and
20, the binned top-down step, first-writer parents, each placement of layer 0,
the finisher (deep paths), graph replays, asynchronous series, modes that
alternate on one workspace, and the wide layer kernel."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import inputs
import oracle
from tests import checks
from tests.test_gpu_single import _check_against_oracle, _gpu_bfs, _small_cases

pytestmark = pytest.mark.gpu

MODES = [dict(td_queue=1), dict(td_queue=2), dict(td_hub_list=1), dict(td_hub_list=2), dict(td_hub_list=3),
         dict(td_hub_list=4), dict(td_queue=1, td_hub_list=1), dict(td_queue=2, td_hub_list=1),
         dict(td_queue=1, td_hub_list=2), dict(td_queue=2, td_hub_list=3)]
MODE_IDS = ["q1", "q2", "hubs", "hubs0", "hubsTD", "hubs01", "q1+hubs", "q2+hubs", "q1+hubs0", "q2+hubsTD"]


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
    return g, hyb.Graph.from_csr(g), inputs.workload_roots("kron16", g, 4)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_edge_case_graphs(torch, hyb, mode):
    for name, g, roots in _small_cases():
        G = hyb.Graph.from_csr(g)
        for rule in ("edges", "td", "bu", "table"):
            for r in roots:
                _say(name, rule, r, mode)
                lv, pa, st = _gpu_bfs(torch, G, r, rule=rule, **mode)
                _check_against_oracle(g, r, lv, pa, st, rule)
        G.close()


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("rule", ["edges", "td", "bu", "table"])
def test_kron16_rules(torch, kron16, rule, mode):
    g, G, roots = kron16
    for r in roots:
        _say("kron16", rule, int(r), mode)
        lv, pa, st = _gpu_bfs(torch, G, int(r), rule=rule, **mode)
        _check_against_oracle(g, int(r), lv, pa, st, rule)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_kron16_alpha_beta_and_task_sizes(torch, kron16, mode):
    g, G, roots = kron16
    r = int(roots[1])
    for a, b, wpw, grid in [(1, 1, 1, 0), (2, 100, 64, 7), (48, 24, 4, 0), (1000, 2, 0, 33)]:
        _say("kron16 alpha/beta", a, b, wpw, grid, mode)
        lv, pa, st = _gpu_bfs(torch, G, r, alpha=a, beta=b, words_per_wave=wpw, grid_blocks=grid, **mode)
        _check_against_oracle(g, r, lv, pa, st, "edges", a, b)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_binned_top_down(torch, hyb, kron16, mode):
    """Binned layers: the count and scatter passes enumerate the queue and hub
    list; the reduce kernel appends to the next ones."""
    g, G, roots = kron16
    for rule in ("edges", "td"):
        for r in roots[:2]:
            _say("kron16 binned", rule, int(r), mode)
            lv, pa, st = _gpu_bfs(torch, G, int(r), rule=rule, td_binned=1, **mode)
            _check_against_oracle(g, int(r), lv, pa, st, rule)
    g18 = inputs.kronecker(18)
    G18 = hyb.Graph.from_csr(g18)
    r = int(inputs.pick_roots(g18, 1, 9)[0])
    lv, pa, st = _gpu_bfs(torch, G18, r, td_binned=1, **mode)
    _check_against_oracle(g18, r, lv, pa, st)
    G18.close()


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_first_writer_parents(torch, kron16, mode):
    g, G, roots = kron16
    for rule in ("edges", "td"):
        r = int(roots[0])
        lv, pa, _ = _gpu_bfs(torch, G, r, rule=rule, first_writer=1, **mode)
        elv, _ = oracle.bfs(g, r)
        assert np.array_equal(lv, elv)
        checks.check_bfs_invariants(g, r, lv, pa, canonical=False)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_layer0_placements(torch, hyb, kron16, mode):
    """Layer 0 in the initialisation kernel, in the one-block kernel and in the
    grid kernel each seed the queue and hub list of F_1 (or F_0)."""
    g, G, _ = kron16
    deg = np.diff(g.off)
    order = np.argsort(deg)
    picks = [int(order[-1]), int(order[np.searchsorted(deg[order], 4096, side="right") - 1]),
             int(order[np.searchsorted(deg[order], 1)]), int(order[-1])]
    for r in picks:
        for rule in ("edges", "td"):
            _say("root degree", int(deg[r]), rule, mode)
            lv, pa, st = _gpu_bfs(torch, G, r, rule=rule, **mode)
            _check_against_oracle(g, r, lv, pa, st, rule)
            assert st["layer0_kernel"] == (2 if deg[r] <= 4096 else 0)
    g17 = inputs.kronecker(17)
    G17 = hyb.Graph.from_csr(g17)
    d = np.diff(g17.off)
    roots = [int(v) for v in np.nonzero((d > 0) & (d <= 4096))[0][:2]]
    for grid in (1, 0):
        for r in roots:
            lv, pa, st = _gpu_bfs(torch, G17, r, grid_blocks=grid, rule="td", **mode)
            _check_against_oracle(g17, r, lv, pa, st, "td")
            assert st["layer0_kernel"] == (1 if grid == 1 else 2)
    G17.close()


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_finisher_and_graph_replay(torch, hyb, kron16, mode):
    """Layers beyond the enqueued kernels run in the one-block finisher, which
    appends to and reads the same queues; graph replays alternate roots."""
    g = inputs.path_graph(1000)
    G = hyb.Graph.from_csr(g)
    for r in (0, 500, 999):
        lv, pa, st = _gpu_bfs(torch, G, r, layers_per_launch=3, **mode)
        _check_against_oracle(g, r, lv, pa, st)
    G.close()
    g16, G16, roots = kron16
    for r in list(roots) + list(roots[:2]):
        _say("kron16 replay", int(r), mode)
        lv, pa, st = _gpu_bfs(torch, G16, int(r), graph_launch=1, **mode)
        _check_against_oracle(g16, int(r), lv, pa)
        lv, pa, st = _gpu_bfs(torch, G16, int(r), layers_per_launch=2, **mode)
        _check_against_oracle(g16, int(r), lv, pa, st)


def test_modes_alternate_on_one_workspace(torch, hyb, kron16):
    """Queue modes, hub lists and the plain path in turn on one stream, with
    asynchronous runs between synchronous ones: each run leaves the counters
    and tails the next one starts from."""
    g, G, roots = kron16
    lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
    pa = torch.empty(g.n, dtype=torch.int32, device="cuda")
    seq = [{}] + MODES + [{}, dict(td_queue=-1, td_hub_list=-1)] + MODES[::-1]
    for i, kw in enumerate(seq):
        r = int(roots[i % len(roots)])
        G.run(r, lv, pa, async_=1, **kw)
        G.run(r, lv, pa, async_=1, rule="td", **kw)
    hyb.hybfs.bfs_graph_sync(G.handle, torch.cuda.current_stream().cuda_stream)
    for i, kw in enumerate(seq):
        r = int(roots[i % len(roots)])
        _say("alternate", i, kw)
        a = _gpu_bfs(torch, G, r, **kw)
        _check_against_oracle(g, r, a[0], a[1], a[2])


def test_kron20_sampled_roots(torch, hyb):
    g = inputs.kronecker(20)
    G = hyb.Graph.from_csr(g)
    roots = inputs.workload_roots("kron20", g, 64)
    for mode in MODES:
        for r in (int(roots[0]), int(roots[5])):
            _say("kron20", r, mode)
            lv, pa, st = _gpu_bfs(torch, G, r, **mode)
            _check_against_oracle(g, r, lv, pa, st)
        lv, pa, st = _gpu_bfs(torch, G, int(roots[9]), alpha=48, words_per_wave=4, **mode)
        _check_against_oracle(g, int(roots[9]), lv, pa, st, "edges", 48, 24)
    G.close()


def test_wide_layer_kernel(torch, hyb):
    """From 2^24 vertices the layers run in the wide build of the layer
    kernel; its list build against the oracle."""
    g = inputs.erdos_renyi(1 << 24, 3 << 23, seed=2424)
    G = hyb.Graph.from_csr(g)
    assert G.info().layer_kernel_wide == 1
    r = int(inputs.pick_roots(g, 1, 11)[0])
    for mode in (dict(td_queue=1, td_hub_list=1), dict(td_queue=2)):
        _say("er24", r, mode)
        # alpha_binned = alpha: the direction trace follows the plain edge rule
        lv, pa, st = _gpu_bfs(torch, G, r, alpha_binned=14, **mode)
        _check_against_oracle(g, r, lv, pa, st)
    G.close()
