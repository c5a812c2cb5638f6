"""Asynchronous runs report through bfs_graph_sync: a clean series returns
BFS_OK with every output equal to the oracle's, and a traversal that fails a
device-side check (forced from the host with the library's test hook, which
makes the finisher report the traversal as failed while every kernel runs
normally) is reported once, then the record is clear."""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

import inputs
import oracle

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


def _graph(hyb, g, fail_root=None):
    old = os.environ.pop("HYBFS_TEST_FAIL_ROOT", None)
    try:
        if fail_root is not None:
            os.environ["HYBFS_TEST_FAIL_ROOT"] = str(int(fail_root))
        return hyb.Graph.from_csr(g)
    finally:
        os.environ.pop("HYBFS_TEST_FAIL_ROOT", None)
        if old is not None:
            os.environ["HYBFS_TEST_FAIL_ROOT"] = old


def test_async_series_syncs_clean_and_matches_oracle(torch, hyb):
    g = inputs.kronecker(14)
    roots = [int(r) for r in inputs.pick_roots(g, 6, 2014)]
    G = _graph(hyb, g)
    s = torch.cuda.Stream()
    sp = s.cuda_stream
    outs = []
    for i, r in enumerate(roots):
        _say("async single root", r, "graph_launch", i % 2)
        lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
        pa = torch.empty(g.n, dtype=torch.int32, device="cuda")
        G.run(r, lv, pa, stream=sp, async_=1, graph_launch=i % 2)
        outs.append((r, lv, pa))
    blv = torch.empty((3, g.n), dtype=torch.int32, device="cuda")
    bpa = torch.empty((3, g.n), dtype=torch.int32, device="cuda")
    G.run_batch(roots[:3], blv, bpa, stream=sp, async_=1)
    hyb.hybfs.bfs_graph_sync(G.handle, sp)
    for r, lv, pa in outs:
        elv, epa = oracle.bfs(g, r)
        assert np.array_equal(lv.cpu().numpy(), elv) and np.array_equal(pa.cpu().numpy(), epa), r
    for i, r in enumerate(roots[:3]):
        elv, epa = oracle.bfs(g, r)
        assert np.array_equal(blv[i].cpu().numpy(), elv) and np.array_equal(bpa[i].cpu().numpy(), epa), r
    G.close()


def test_failed_async_runs_are_reported_once(torch, hyb):
    g = inputs.kronecker(12)
    roots = [int(r) for r in inputs.pick_roots(g, 4, 2012)]
    bad = roots[1]
    G = _graph(hyb, g, fail_root=bad)
    s = torch.cuda.Stream()
    sp = s.cuda_stream
    lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
    pa = torch.empty(g.n, dtype=torch.int32, device="cuda")
    HybfsError = hyb.hybfs.HybfsError
    for gl in (0, 1):
        _say("async series with a failing root, graph_launch", gl)
        for r in roots:
            G.run(r, lv, pa, stream=sp, async_=1, graph_launch=gl)
        with pytest.raises(HybfsError) as ei:
            hyb.hybfs.bfs_graph_sync(G.handle, sp)
        assert ei.value.code == hyb.hybfs.BFS_E_DEVICE
        assert "1 asynchronous" in str(ei.value)
        hyb.hybfs.bfs_graph_sync(G.handle, sp)        # reported once: clear now
    # the runs of the other roots are unaffected
    for r in (roots[0], roots[2]):
        G.run(r, lv, pa, stream=sp, async_=1)
        hyb.hybfs.bfs_graph_sync(G.handle, sp)
        elv, epa = oracle.bfs(g, r)
        assert np.array_equal(lv.cpu().numpy(), elv) and np.array_equal(pa.cpu().numpy(), epa)
    # a synchronous run reports its own failure at once and leaves no record
    with pytest.raises(HybfsError) as ei:
        G.run(bad, lv, pa, stream=sp)
    assert ei.value.code == hyb.hybfs.BFS_E_DEVICE
    hyb.hybfs.bfs_graph_sync(G.handle, sp)
    # a batch holding the failing root, asynchronously
    blv = torch.empty((4, g.n), dtype=torch.int32, device="cuda")
    bpa = torch.empty((4, g.n), dtype=torch.int32, device="cuda")
    _say("async batch with a failing root")
    G.run_batch(roots, blv, bpa, stream=sp, async_=1)
    with pytest.raises(HybfsError) as ei:
        hyb.hybfs.bfs_graph_sync(G.handle, sp)
    assert ei.value.code == hyb.hybfs.BFS_E_DEVICE
    hyb.hybfs.bfs_graph_sync(G.handle, sp)
    G.close()
