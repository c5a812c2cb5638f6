"""bfs_run_noalloc (the entry point that allocates no device memory: its
scratch is the library's fixed device array) against bfs_run, through the
C ABI: two calls in a row, the second on a smaller graph, outputs and
per-layer statistics equal byte for byte; a graph above the array's limit and
host outputs are refused."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import inputs

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


def _both(torch, G, g, root, **kw):
    lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
    pa = torch.empty(g.n, dtype=torch.int32, device="cuda")
    _, _, st = G.run(root, lv, pa, stats=True, **kw)
    nlv = torch.full((g.n,), 7, dtype=torch.int32, device="cuda")
    npa = torch.full((g.n,), 7, dtype=torch.int32, device="cuda")
    _, _, nst = G.run_noalloc(root, nlv, npa, stats=True, **kw)
    torch.cuda.synchronize()
    return lv, pa, st, nlv, npa, nst


def _layers(st):
    return [(r["dir"], r["n_f"], r["m_f"], r["m_u"], r["v_u"]) for r in st["layers"]]


def test_noalloc_equals_bfs_run_two_calls_second_smaller(torch, hyb):
    big = inputs.kronecker(16)
    small = inputs.kronecker(11)
    for g, label in ((big, "kron16"), (small, "kron11")):
        G = hyb.Graph.from_csr(g)
        for root in [int(r) for r in inputs.pick_roots(g, 2, 77)]:
            _say("noalloc vs bfs_run:", label, "root", root)
            lv, pa, st, nlv, npa, nst = _both(torch, G, g, root)
            assert torch.equal(lv, nlv) and torch.equal(pa, npa)
            assert nst["num_layers"] == st["num_layers"] and nst["reached"] == st["reached"]
            assert nst["reached_degree_sum"] == st["reached_degree_sum"]
            assert _layers(nst) == _layers(st)
        G.close()


def test_noalloc_options_and_edge_graphs(torch, hyb):
    # forced directions and a deep path (layers beyond the launch depth run in
    # the finisher), one after another on the shared array
    g = inputs.kronecker(13)
    G = hyb.Graph.from_csr(g)
    root = int(inputs.pick_roots(g, 1, 5)[0])
    for kw in ({"rule": "td"}, {"rule": "bu"}, {"rule": "table"}, {"alpha": 48, "words_per_wave": 4},
               {"td_binned": 1}):
        _say("noalloc options", kw)
        lv, pa, _, nlv, npa, _ = _both(torch, G, g, root, **kw)
        assert torch.equal(lv, nlv) and torch.equal(pa, npa)
    G.close()
    n = 3000
    off = np.zeros(n + 1, np.int64)
    cols = []
    for v in range(n):
        nb = [u for u in (v - 1, v + 1) if 0 <= u < n]
        cols.extend(nb)
        off[v + 1] = off[v] + len(nb)
    P = hyb.Graph(off, np.array(cols, np.int32))
    _say("noalloc path of", n)
    lv = torch.empty(n, dtype=torch.int32, device="cuda")
    pa = torch.empty(n, dtype=torch.int32, device="cuda")
    P.run_noalloc(17, lv, pa)
    torch.cuda.synchronize()
    idx = np.arange(n)
    assert np.array_equal(lv.cpu().numpy(), np.abs(idx - 17))
    exp_par = np.where(idx < 17, idx + 1, np.where(idx > 17, idx - 1, 17))
    assert np.array_equal(pa.cpu().numpy(), exp_par)
    P.close()


def test_noalloc_refuses_host_outputs_and_async(torch, hyb):
    g = inputs.kronecker(8)
    G = hyb.Graph.from_csr(g)
    h = np.empty(g.n, np.int32)
    opt = hyb.hybfs.bfs_options_init(out_on_device=0)
    rc = hyb.hybfs.load().bfs_run_noalloc(G.handle, 0, h.ctypes.data, h.ctypes.data, opt, None)
    assert rc == hyb.hybfs.BFS_E_INVALID
    lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
    opt = hyb.hybfs.bfs_options_init(out_on_device=1)
    opt.async_ = 1
    rc = hyb.hybfs.load().bfs_run_noalloc(G.handle, 0, lv.data_ptr(), lv.data_ptr(), opt, None)
    assert rc == hyb.hybfs.BFS_E_INVALID
    G.close()
