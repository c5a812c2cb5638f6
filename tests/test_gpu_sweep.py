"""Parity on the shape of the paper's SCALE x edgefactor sweep (Section 8,
Figure 3: Kronecker graphs at edgefactor 16, 32 and 64): Kronecker SCALE 16
and 18 at edgefactor 32 and 64, several roots each, levels and canonical
parents byte-exact against the oracle and the per-layer counters and
direction trace equal to the oracle's replay; default and tuned-style
options, every direction rule on one graph."""
from __future__ import annotations

import sys

import pytest

import inputs
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


@pytest.mark.parametrize("scale,ef", [(16, 32), (16, 64), (18, 32), (18, 64)])
def test_kronecker_edgefactor(torch, hyb, scale, ef):
    g = inputs.kronecker(scale, ef, seed=5000 + 100 * ef + scale)
    G = hyb.Graph.from_csr(g)
    roots = [int(r) for r in inputs.pick_roots(g, 4, 6000 + scale + ef)]
    for r in roots:
        _say(f"kron{scale} ef{ef} root {r}")
        lv, pa, st = _gpu_bfs(torch, G, r)
        _check_against_oracle(g, r, lv, pa, st)
    r = roots[0]
    lv, pa, st = _gpu_bfs(torch, G, r, alpha=48, words_per_wave=4)
    _check_against_oracle(g, r, lv, pa, st, "edges", 48, 24)
    if scale == 16:
        for rule in ("td", "bu", "table"):
            _say(f"kron{scale} ef{ef} rule {rule}")
            lv, pa, st = _gpu_bfs(torch, G, r, rule=rule)
            _check_against_oracle(g, r, lv, pa, st, rule)
    G.close()
