"""Per-layer work counts (option count_work) against what the oracle fixes:
outputs unchanged; a top-down layer examines exactly its frontier's edges
and discovers exactly the next frontier; a bottom-up layer examines exactly
the unvisited vertices of nonzero degree (the oracle's candidates), finds
exactly the next frontier, and probes at least the entries Algorithm 2 reads
before each first hit (the oracle's sum of s_v) and at most that plus what
the 64-wide phase-2 steps read past a hit."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import inputs
import oracle
from tests.test_gpu_single import _check_against_oracle, _gpu_bfs

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


def _check_counts(g, root, st, probe_k_serial):
    elv, _ = oracle.bfs(g, root)
    rep = oracle.layer_replay(g, elv)
    L = len(rep["n_f"])
    for d, lay in enumerate(st["layers"][:L]):
        w = lay["work"]
        nxt = int(rep["n_f"][d + 1]) if d + 1 < L else 0
        if d == 0 and st["layer0_kernel"] != 0:
            assert w == [0] * 6          # layer 0 ran outside the layer kernel
            continue
        if lay["dir"] == 0:
            assert w[0] == lay["m_f"], (d, w)
            assert w[3] == nxt, (d, w)
            assert w[1] >= w[3] and w[2] >= w[3]
        else:
            s_sum, cands = oracle.bottom_up_probes(g, elv, d)
            assert w[0] == cands, (d, w, cands)
            assert w[5] == nxt, (d, w)
            probed = w[1] + w[4]
            assert probed >= s_sum, (d, w, s_sum)
            # phase 2 reads whole 64-entry steps; probes issued together (not
            # serial) may read up to three entries past a hit in each phase-1 round
            assert probed <= s_sum + 63 * w[3] + (0 if probe_k_serial else 6 * w[0]), (d, w, s_sum)


@pytest.mark.parametrize("rule", ["edges", "td", "bu", "table"])
def test_work_counts_kron16(torch, hyb, rule):
    g = inputs.kronecker(16)
    G = hyb.Graph.from_csr(g)
    for r in inputs.workload_roots("kron16", g, 4):
        r = int(r)
        for serial in (1, -1):
            _say("kron16 counts", rule, r, serial)
            lv, pa, st = _gpu_bfs(torch, G, r, rule=rule, count_work=1, bu_serial_probes=serial)
            _check_against_oracle(g, r, lv, pa, st, rule)
            _check_counts(g, r, st, serial == 1)
    G.close()


def test_work_counts_edge_graphs_and_kron20(torch, hyb):
    for g, roots in ((inputs.path_graph(300), [0, 150]), (inputs.star_graph(300, center=5), [5, 17]),
                     (inputs.grid_graph(40, 30), [0, 611])):
        G = hyb.Graph.from_csr(g)
        for r in roots:
            lv, pa, st = _gpu_bfs(torch, G, r, count_work=1, layers_per_launch=3, bu_serial_probes=1)
            _check_against_oracle(g, r, lv, pa, st)
            _check_counts(g, r, st, True)
        G.close()
    g = inputs.kronecker(20)
    G = hyb.Graph.from_csr(g)
    r = int(inputs.workload_roots("kron20", g, 64)[3])
    lv, pa, st = _gpu_bfs(torch, G, r, count_work=1)
    _check_against_oracle(g, r, lv, pa, st)
    _check_counts(g, r, st, False)
    G.close()
