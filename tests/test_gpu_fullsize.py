"""Parity at the full workload sizes, in the configuration the benchmark
times: Kronecker SCALE 26 (67M vertices, 2.1G stored entries) single-root
traversals with the default options, byte-exact against the oracle for two
roots (among them the root whose sparse-frontier bottom-up layer scans long
rows); and a SCALE-22 batch of 64 roots, every row equal to the single-root
run of its root and two rows equal to the oracle."""
from __future__ import annotations

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


def test_kron26_two_roots_byte_exact(torch, hyb):
    _say("generating Kronecker SCALE 26")
    g = inputs.workload_graph("kron26")
    roots = inputs.workload_roots("kron26", g, 64)
    G = hyb.Graph.from_csr(g, flags=hyb.hybfs.BFS_GRAPH_ASSUME_VALID)
    lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
    pa = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for r in (int(roots[0]), int(roots[1])):
        _, _, st = G.run(r, lv, pa, stats=True)
        torch.cuda.synchronize()
        _say("kron26 root", r, "layers", st["num_layers"], "reached", st["reached"])
        elv, epa = oracle.bfs(g, r)
        got_l = lv.cpu().numpy()
        bad = np.nonzero(got_l != elv)[0]
        assert len(bad) == 0, f"root {r}: level mismatch at {bad[:8]}"
        got_p = pa.cpu().numpy()
        bad = np.nonzero(got_p != epa)[0]
        assert len(bad) == 0, f"root {r}: parent mismatch at {bad[:8]}"
        assert st["reached"] == int((elv >= 0).sum())
        assert st["num_layers"] == int(elv.max()) + 1
        del elv, epa, got_l, got_p
    G.close()


def test_kron22_batch_of_64_equals_single_runs(torch, hyb):
    g = inputs.workload_graph("kron22")
    roots = inputs.workload_roots("kron22", g, 64).astype(np.int32)
    G = hyb.Graph.from_csr(g)
    k = len(roots)
    blv = torch.empty((k, g.n), dtype=torch.int32, device="cuda")
    bpa = torch.empty((k, g.n), dtype=torch.int32, device="cuda")
    G.run_batch(roots, blv, bpa)
    lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
    pa = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for i, r in enumerate(roots):
        G.run(int(r), lv, pa)
        torch.cuda.synchronize()
        assert torch.equal(blv[i], lv) and torch.equal(bpa[i], pa), f"row {i} (root {int(r)})"
    _say("kron22 batch rows equal single runs")
    for i in (0, 63):
        elv, epa = oracle.bfs(g, int(roots[i]))
        assert np.array_equal(blv[i].cpu().numpy(), elv) and np.array_equal(bpa[i].cpu().numpy(), epa), i
    G.close()
