"""Serving (bfs_serve_*) on the GPU: a burst of queries over six resident
graphs of uneven size is answered exactly as each query alone (bfs_run) and
as the oracle; host outputs; admission under a small memory budget; a paced
stream; error codes."""
from __future__ import annotations

import sys
import time

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


@pytest.fixture(scope="module")
def graphs(hyb):
    gs = [inputs.kronecker(10), inputs.kronecker(12), inputs.kronecker(14), inputs.kronecker(16),
          inputs.erdos_renyi(1 << 14, 4 << 14, seed=3014), inputs.path_graph(3000)]
    Gs = [hyb.Graph.from_csr(g) for g in gs]
    return gs, Gs


def _queries(gs, count, seed):
    rng = np.random.default_rng(seed)
    w = np.array([g.n for g in gs], dtype=np.float64)
    w /= w.sum()
    out = []
    for _ in range(count):
        gi = int(rng.choice(len(gs), p=w))
        live = np.nonzero(np.diff(gs[gi].off) > 0)[0]
        out.append((gi, int(rng.choice(live))))
    return out


def _alone(torch, G, root):
    lv = torch.empty(G.n, dtype=torch.int32, device="cuda")
    pa = torch.empty(G.n, dtype=torch.int32, device="cuda")
    G.run(root, lv, pa)
    torch.cuda.synchronize()
    return lv.cpu().numpy(), pa.cpu().numpy()


def test_burst_mix_equals_alone(torch, hyb, graphs):
    gs, Gs = graphs
    # batch whenever two or more queries of a graph are queued
    S = hyb.hybfs.Server(streams=4, max_batch=64, batch_threshold=2)
    ids = [S.add_graph(G) for G in Gs]
    qs = _queries(gs, 400, 1)
    bufs, tickets = [], []
    for gi, r in qs:
        lv = torch.empty(gs[gi].n, dtype=torch.int32, device="cuda")
        pa = torch.empty(gs[gi].n, dtype=torch.int32, device="cuda")
        bufs.append((lv, pa))
        tickets.append(S.submit(ids[gi], r, lv.data_ptr(), pa.data_ptr()))
    for t in tickets:
        S.wait(t, 60_000_000)
    st = S.stats()
    _say("burst stats", st)
    assert st["completed"] == len(qs) and st["failed"] == 0
    assert st["batched_requests"] > 0 and st["batches"] < len(qs)
    assert 0 < st["p50_us"] <= st["p99_us"] <= st["max_us"]
    assert st["running"] == 0 and st["queued"] == 0
    # what stays charged is what the slots keep cached for the next queries
    assert 0 < st["bytes_in_use"] <= st["peak_bytes"] <= st["memory_budget"]
    alone = {}
    te = 0.0
    for (gi, r), (lv, pa) in zip(qs, bufs):
        key = (gi, r)
        if key not in alone:
            alone[key] = _alone(torch, Gs[gi], r)
        elv, epa = alone[key]
        assert np.array_equal(lv.cpu().numpy(), elv), key
        assert np.array_equal(pa.cpu().numpy(), epa), key
        te += oracle.traversed_edges(gs[gi], elv)
    assert abs(st["traversed_edges"] - te) < 0.5
    for gi, r in list(alone)[:12]:
        olv, opa = oracle.bfs(gs[gi], r)
        assert np.array_equal(alone[(gi, r)][0], olv) and np.array_equal(alone[(gi, r)][1], opa)
    S.close()


def test_host_outputs(torch, hyb, graphs):
    gs, Gs = graphs
    S = hyb.hybfs.Server(streams=2, out_on_device=0)
    ids = [S.add_graph(G) for G in Gs]
    qs = _queries(gs, 40, 2)
    bufs, tickets = [], []
    for gi, r in qs:
        lv = np.full(gs[gi].n, 7, dtype=np.int32)
        pa = np.full(gs[gi].n, 7, dtype=np.int32)
        bufs.append((lv, pa))
        tickets.append(S.submit(ids[gi], r, lv.ctypes.data, pa.ctypes.data))
    for t in tickets:
        S.wait(t)
    for (gi, r), (lv, pa) in zip(qs, bufs):
        olv, opa = oracle.bfs(gs[gi], r)
        assert np.array_equal(lv, olv) and np.array_equal(pa, opa), (gi, r)
    S.close()


def test_small_budget_forces_admission_waits(torch, hyb, graphs):
    gs, Gs = graphs
    from paper_1704_02259_amd import hybfs
    # room for one single-root traversal of the SCALE-16 graph (workspace and
    # host-output staging) at a time: the other slots have to wait
    g16 = gs[3]
    budget = int(Gs[3].info().workspace_bytes + g16.n * 8 + 4096)
    S = hyb.hybfs.Server(streams=4, max_batch=8, out_on_device=0, memory_budget=budget)
    gid = S.add_graph(Gs[3])
    live = np.nonzero(np.diff(g16.off) > 0)[0]
    roots = [int(x) for x in np.random.default_rng(3).choice(live, 48)]
    bufs = [(np.empty(g16.n, np.int32), np.empty(g16.n, np.int32)) for _ in roots]
    tickets = [S.submit(gid, r, lv.ctypes.data, pa.ctypes.data) for r, (lv, pa) in zip(roots, bufs)]
    for t in tickets:
        S.wait(t)
    st = S.stats()
    _say("budget stats", st)
    assert st["completed"] == len(roots)
    assert st["peak_bytes"] <= budget
    assert st["admission_waits"] > 0
    for r, (lv, pa) in zip(roots[:8], bufs[:8]):
        olv, opa = oracle.bfs(g16, r)
        assert np.array_equal(lv, olv) and np.array_equal(pa, opa)
    S.close()
    # a budget below any query's footprint: the query fails, the server stays usable
    S = hyb.hybfs.Server(streams=1, memory_budget=1024)
    gid = S.add_graph(Gs[3])
    lv = torch.empty(g16.n, dtype=torch.int32, device="cuda")
    t = S.submit(gid, roots[0], lv.data_ptr(), lv.data_ptr())
    with pytest.raises(hybfs.HybfsError) as ei:
        S.wait(t)
    assert ei.value.code == hybfs.BFS_E_NOMEM
    assert S.stats()["failed"] == 1
    S.close()


def _device_used(torch):
    free, total = torch.cuda.mem_get_info()
    return total - free


def test_cached_workspaces_stay_within_budget(torch, hyb, graphs):
    """A traversal leaves its workspaces cached with the graph for its slot's
    stream; on a graph of 2^23 vertices they include the binned top-down
    buckets (hundreds of MiB).  Two such graphs and a small one, three slots
    and a budget of 1.5 such footprints: caches for both large graphs would
    exceed it, so a slot that moves from one to the other must release an idle
    cache or wait.  The charged peak stays within the budget, so does the
    device memory actually allocated (sampled while the queries run), and
    destroying the server gives it back."""
    gs, Gs = graphs
    big = [inputs.erdos_renyi(1 << 23, 1 << 24, seed=2323 + i) for i in range(2)]
    Gbig = [hyb.Graph.from_csr(g) for g in big]
    g16, G16 = gs[3], Gs[3]
    lives = [np.nonzero(np.diff(g.off) > 0)[0] for g in big + [g16]]
    rng = np.random.default_rng(23)
    _alone(torch, G16, int(lives[2][0]))     # kernels loaded before memory is measured
    slack = 64 << 20                         # allocation granularity, streams' own buffers

    # one slot, one query: the charge is what the traversal left allocated
    lv = torch.empty(big[0].n, dtype=torch.int32, device="cuda")
    pa = torch.empty(big[0].n, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    S = hyb.hybfs.Server(streams=1)
    gid = S.add_graph(Gbig[0])
    u0 = _device_used(torch)
    S.wait(S.submit(gid, int(lives[0][0]), lv.data_ptr(), pa.data_ptr()))
    held = S.stats()["bytes_in_use"]
    grew = _device_used(torch) - u0
    _say("one query holds", held, "device grew by", grew)
    assert held > Gbig[0].info().workspace_bytes + (128 << 20)    # the binned buckets are charged
    assert 0.9 * held <= grew <= held + slack
    S.close()
    assert _device_used(torch) - u0 <= slack                     # destroy released the caches

    budget = int(1.5 * held)
    S = hyb.hybfs.Server(streams=3, max_batch=4, batch_threshold=2, memory_budget=budget)
    Gall = Gbig + [G16]
    ids = [S.add_graph(G) for G in Gall]
    qs = [(i % 3, int(rng.choice(lives[i % 3]))) for i in range(36)]
    bufs = []
    for gi, r in qs:
        n = Gall[gi].n
        bufs.append((torch.empty(n, dtype=torch.int32, device="cuda"),
                     torch.empty(n, dtype=torch.int32, device="cuda")))
    torch.cuda.synchronize()
    u0 = _device_used(torch)
    tickets = [S.submit(ids[gi], r, lv.data_ptr(), pa.data_ptr()) for (gi, r), (lv, pa) in zip(qs, bufs)]
    pending, most = set(tickets), 0
    deadline = time.time() + 120
    while pending and time.time() < deadline:
        most = max(most, _device_used(torch) - u0)
        for t in list(pending):
            if S.poll(t):
                pending.discard(t)
    assert not pending
    st = S.stats()
    _say("cached-workspace stats", st, "sampled device growth", most)
    assert st["completed"] == len(qs) and st["failed"] == 0
    assert st["peak_bytes"] <= budget
    assert st["evictions"] > 0
    assert most <= budget + slack
    for (gi, r), (lv, pa) in list(zip(qs, bufs))[:9]:
        elv, epa = _alone(torch, Gall[gi], r)
        assert np.array_equal(lv.cpu().numpy(), elv) and np.array_equal(pa.cpu().numpy(), epa), (gi, r)
    olv, opa = oracle.bfs(big[1], qs[1][1])
    assert np.array_equal(bufs[1][0].cpu().numpy(), olv) and np.array_equal(bufs[1][1].cpu().numpy(), opa)
    S.close()
    del bufs
    for G in Gbig:
        G.close()


def test_host_output_batches_share_a_small_budget(torch, hyb, graphs):
    """Host outputs: a batch of k roots stages its outputs in an 8·k·n-byte
    device buffer that its slot keeps.  Two slots taking batches of up to 8
    under a budget of 1.5 batch footprints must release each other's idle
    staging and workspaces or wait; every answer still equals the oracle's."""
    gs, Gs = graphs
    g16, G16 = gs[3], Gs[3]
    info = G16.info()
    batch = info.batch_workspace_bytes + 8 * 8 * g16.n
    single = info.workspace_bytes + (g16.n + 64) * 8
    budget = int(1.5 * max(batch, single))
    S = hyb.hybfs.Server(streams=2, max_batch=8, batch_threshold=2, out_on_device=0, memory_budget=budget)
    gid = S.add_graph(G16)
    live = np.nonzero(np.diff(g16.off) > 0)[0]
    roots = [int(x) for x in np.random.default_rng(16).choice(live, 64)]
    bufs = [(np.full(g16.n, 7, np.int32), np.full(g16.n, 7, np.int32)) for _ in roots]
    tickets = [S.submit(gid, r, lv.ctypes.data, pa.ctypes.data) for r, (lv, pa) in zip(roots, bufs)]
    for t in tickets:
        S.wait(t)
    st = S.stats()
    _say("host-output batch stats", st)
    assert st["completed"] == len(roots) and st["failed"] == 0
    assert st["batched_requests"] > 0
    assert st["peak_bytes"] <= budget
    for r, (lv, pa) in zip(roots, bufs):
        olv, opa = oracle.bfs(g16, r)
        assert np.array_equal(lv, olv) and np.array_equal(pa, opa), r
    S.close()


def test_paced_stream_and_poll(torch, hyb, graphs):
    gs, Gs = graphs
    S = hyb.hybfs.Server(streams=3)
    ids = [S.add_graph(G) for G in Gs]
    qs = _queries(gs, 120, 4)
    gaps = np.random.default_rng(4242).exponential(200e-6, len(qs))
    bufs, tickets = [], []
    for (gi, r), gap in zip(qs, gaps):
        time.sleep(gap)
        lv = torch.empty(gs[gi].n, dtype=torch.int32, device="cuda")
        pa = torch.empty(gs[gi].n, dtype=torch.int32, device="cuda")
        bufs.append((lv, pa))
        tickets.append(S.submit(ids[gi], r, lv.data_ptr(), pa.data_ptr()))
    pending = set(tickets)
    deadline = time.time() + 60
    while pending and time.time() < deadline:
        for t in list(pending):
            if S.poll(t):
                pending.discard(t)
    assert not pending
    alone = {}
    for (gi, r), (lv, pa) in zip(qs, bufs):
        if (gi, r) not in alone:
            alone[(gi, r)] = _alone(torch, Gs[gi], r)
        assert np.array_equal(lv.cpu().numpy(), alone[(gi, r)][0])
        assert np.array_equal(pa.cpu().numpy(), alone[(gi, r)][1])
    S.close()


def test_error_codes(torch, hyb, graphs):
    from paper_1704_02259_amd import hybfs
    gs, Gs = graphs
    S = hyb.hybfs.Server(streams=1, queue_capacity=1)
    gid = S.add_graph(Gs[3])
    lv = torch.empty(gs[3].n, dtype=torch.int32, device="cuda")
    pa = torch.empty(gs[3].n, dtype=torch.int32, device="cuda")
    for args, code in (((gid + 5, 0), hybfs.BFS_E_NOTFOUND), ((gid, gs[3].n), hybfs.BFS_E_INVALID),
                       ((gid, -1), hybfs.BFS_E_INVALID)):
        with pytest.raises(hybfs.HybfsError) as ei:
            S.submit(args[0], args[1], lv.data_ptr(), pa.data_ptr())
        assert ei.value.code == code
    live = int(np.nonzero(np.diff(gs[3].off) > 0)[0][0])
    t = S.submit(gid, live, lv.data_ptr(), pa.data_ptr())
    with pytest.raises(hybfs.HybfsError) as ei:
        S.submit(gid, live, lv.data_ptr(), pa.data_ptr())
    assert ei.value.code == hybfs.BFS_E_BUSY
    S.wait(t)
    with pytest.raises(hybfs.HybfsError) as ei:
        S.wait(t)
    assert ei.value.code == hybfs.BFS_E_NOTFOUND
    S.reset_stats()
    assert S.stats()["completed"] == 0
    S.close()
