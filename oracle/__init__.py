"""CPU oracle -- test infrastructure only.

Plain serial C (``bfs_oracle.c``) behind ctypes.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package; the GPU library never links, loads or calls it, and the two share
no code.  Inputs come from the separate ``inputs`` module.

Functions and the passage each follows:
  bfs                 -- Section 4 (layers, predecessor array P), with the
                         canonical smallest-id parent fixing the tree that
                         Section 7.1 says a parallel run leaves open.
  layer_replay        -- Section 4 heuristic inputs v_f, e_f, e_u per layer.
  direction_trace     -- Algorithm 3 as a state machine; rule "table" is the
                         reading that reproduces Table 2.
  traversed_edges     -- TEPS numerator, Section 6.3.
  bottom_up_probes    -- entries Algorithm 2 reads in one layer.
  algorithmic_bytes   -- compulsory traffic of a BFS at element granularity
                         (cost model built on Algorithms 1 and 2, see the
                         function's docstring).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bfs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

RULES = {"beamer": 0, "table": 1, "td": 2, "bu": 3}
TOP_DOWN, BOTTOM_UP = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle (plain gcc -O3: compiler optimisation only, the C
    source itself is a plain serial loop nest)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.oracle_bfs.restype = ctypes.c_int
    lib.oracle_bfs.argtypes = [i64, vp, vp, i32, vp, vp]
    lib.oracle_bfs_levels.restype = ctypes.c_int
    lib.oracle_bfs_levels.argtypes = [i64, vp, vp, i32, vp]
    lib.oracle_canonical_parents.restype = ctypes.c_int
    lib.oracle_canonical_parents.argtypes = [i64, vp, vp, i32, vp, vp]
    lib.oracle_layer_replay.restype = i64
    lib.oracle_layer_replay.argtypes = [i64, vp, vp, i64, vp, vp, vp, vp]
    lib.oracle_direction_trace.restype = ctypes.c_int
    lib.oracle_direction_trace.argtypes = [ctypes.c_int, i64, i64, i64, i64, vp, vp, vp, vp, vp]
    lib.oracle_reached_degree_sum.restype = i64
    lib.oracle_reached_degree_sum.argtypes = [i64, vp, vp]
    lib.oracle_bottom_up_probes.restype = i64
    lib.oracle_bottom_up_probes.argtypes = [i64, vp, vp, vp, i32, vp]
    _lib = lib
    return lib


def _csr(g):
    off = np.ascontiguousarray(g.off, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.int32)
    return off, col


def bfs(g, root: int) -> tuple[np.ndarray, np.ndarray]:
    """Levels (hop distance, -1 unreached) and canonical parents."""
    off, col = _csr(g)
    level = np.empty(g.n, dtype=np.int32)
    parent = np.empty(g.n, dtype=np.int32)
    rc = _load().oracle_bfs(g.n, off.ctypes.data, col.ctypes.data, int(root),
                            level.ctypes.data, parent.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle_bfs failed rc={rc}")
    return level, parent


def canonical_parents(g, root: int, level: np.ndarray) -> np.ndarray:
    off, col = _csr(g)
    level = np.ascontiguousarray(level, dtype=np.int32)
    parent = np.empty(g.n, dtype=np.int32)
    rc = _load().oracle_canonical_parents(g.n, off.ctypes.data, col.ctypes.data, int(root),
                                          level.ctypes.data, parent.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_canonical_parents failed")
    return parent


def layer_replay(g, level: np.ndarray) -> dict:
    """Per-layer n_f, m_f, m_u, v_u (arrays of length L = deepest level + 1)."""
    level = np.ascontiguousarray(level, dtype=np.int32)
    L = int(level.max()) + 1 if level.size else 0
    cap = max(L, 1)
    arrs = {k: np.zeros(cap, dtype=np.int64) for k in ("n_f", "m_f", "m_u", "v_u")}
    got = _load().oracle_layer_replay(g.n, np.ascontiguousarray(g.off).ctypes.data,
                                      level.ctypes.data, cap,
                                      arrs["n_f"].ctypes.data, arrs["m_f"].ctypes.data,
                                      arrs["m_u"].ctypes.data, arrs["v_u"].ctypes.data)
    if got != L:
        raise RuntimeError(f"oracle_layer_replay returned {got} layers, expected {L}")
    return {k: v[:L] for k, v in arrs.items()}


def direction_trace(rule: str, n: int, rep: dict, alpha: int = 14, beta: int = 24) -> np.ndarray:
    """Direction of each layer, 0 = top-down, 1 = bottom-up."""
    L = len(rep["n_f"])
    dirs = np.zeros(max(L, 1), dtype=np.int32)
    a = {k: np.ascontiguousarray(rep[k], dtype=np.int64) for k in ("n_f", "m_f", "m_u", "v_u")}
    rc = _load().oracle_direction_trace(RULES[rule], alpha, beta, n, L,
                                        a["n_f"].ctypes.data, a["m_f"].ctypes.data,
                                        a["m_u"].ctypes.data, a["v_u"].ctypes.data,
                                        dirs.ctypes.data)
    if rc != 0:
        raise ValueError(rule)
    return dirs[:L]


def reached_degree_sum(g, level: np.ndarray) -> int:
    level = np.ascontiguousarray(level, dtype=np.int32)
    return int(_load().oracle_reached_degree_sum(g.n, np.ascontiguousarray(g.off).ctypes.data,
                                                 level.ctypes.data))


def traversed_edges(g, level: np.ndarray) -> float:
    """TEPS numerator: undirected edges inside the reached component (half of
    the directed CSR entries of the reached vertices)."""
    return reached_degree_sum(g, level) / 2.0


def bottom_up_probes(g, level: np.ndarray, d: int) -> tuple[int, int]:
    """(sum over candidates of entries read before the first hit, #candidates)."""
    off, col = _csr(g)
    level = np.ascontiguousarray(level, dtype=np.int32)
    cnt = ctypes.c_int64(0)
    s = _load().oracle_bottom_up_probes(g.n, off.ctypes.data, col.ctypes.data,
                                        level.ctypes.data, int(d), ctypes.byref(cnt))
    return int(s), int(cnt.value)


def algorithmic_bytes(g, level: np.ndarray, rep: dict | None = None) -> dict:
    """Compulsory HBM traffic of one BFS at element granularity.

    With F_d the layers, per layer d that has a frontier the cheaper of
      top-down  (Algorithm 1): 16|F_d| (two int64 row offsets per frontier
                vertex) + 4*sum deg(F_d) (int32 columns) + 4|F_d| + 4|F_{d+1}|
                (queue in and out)
      bottom-up (Algorithm 2): 3*ceil(n/8) (visited, frontier, next bitmaps)
                + 8|U'_d| (row offsets of the candidates) + 4*sum s_v(d)
                (columns read up to the first frontier hit), U'_d = vertices of
                nonzero degree not in layers 0..d
    plus 8n for writing level and parent once.
    """
    if rep is None:
        rep = layer_replay(g, level)
    n = g.n
    L = len(rep["n_f"])
    per_layer = []
    total = 8 * n
    for d in range(L):
        nf = int(rep["n_f"][d])
        if nf == 0:
            continue
        nf_next = int(rep["n_f"][d + 1]) if d + 1 < L else 0
        td = 16 * nf + 4 * int(rep["m_f"][d]) + 4 * nf + 4 * nf_next
        s, cnt = bottom_up_probes(g, level, d)
        bu = 3 * ((n + 7) // 8) + 8 * cnt + 4 * s
        per_layer.append((td, bu))
        total += min(td, bu)
    return {"bytes": total, "per_layer": per_layer}
