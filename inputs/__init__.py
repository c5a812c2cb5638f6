"""Seeded synthetic graph inputs shared by the oracle, the tests and the bench.

Holds no breadth-first-search arithmetic: it only builds CSR graphs (int64 row
offsets, int32 ascending column indices, symmetric, no self-loops or duplicate
entries) and draws roots.  The Kronecker recipe follows the Graph500-style
generator the paper uses (Section 6.2: SCALE, edgefactor, initiator
A=0.57 B=0.19 C=0.19 D=0.05, bidirectional edges); the exact edge set is our
own seeded stream, not Graph500's.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None

KRON_A, KRON_B, KRON_C = 0.57, 0.19, 0.19


def build(force: bool = True) -> str:
    """Compile the generator shared library in place (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    vp, i64, u64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
    lib.gg_kronecker.restype = vp
    lib.gg_kronecker.argtypes = [i32, i32, u64, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, i32]
    lib.gg_erdos_renyi.restype = vp
    lib.gg_erdos_renyi.argtypes = [i64, i64, u64, i32]
    lib.gg_num_vertices.restype = i64
    lib.gg_num_vertices.argtypes = [vp]
    lib.gg_nnz.restype = i64
    lib.gg_nnz.argtypes = [vp]
    lib.gg_emit.restype = i32
    lib.gg_emit.argtypes = [vp, vp, vp, i32]
    lib.gg_free.restype = None
    lib.gg_free.argtypes = [vp]
    lib.gg_pick_roots.restype = i64
    lib.gg_pick_roots.argtypes = [i64, vp, u64, i64, vp]
    lib.gg_set_verbose.restype = None
    lib.gg_set_verbose.argtypes = [i32]
    lib.gg_uniform_u64.restype = None
    lib.gg_uniform_u64.argtypes = [u64, u64, i64, vp]
    _lib = lib
    return lib


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _emit(state) -> tuple[np.ndarray, np.ndarray]:
    lib = _load()
    if not state:
        raise MemoryError("graph generation failed")
    try:
        n = lib.gg_num_vertices(state)
        nnz = lib.gg_nnz(state)
        off = np.empty(n + 1, dtype=np.int64)
        col = np.empty(max(nnz, 0), dtype=np.int32)
        rc = lib.gg_emit(state, off.ctypes.data, col.ctypes.data if nnz else None, _threads())
        if rc != 0:
            raise RuntimeError("gg_emit failed")
    finally:
        lib.gg_free(state)
    return off, col


@dataclass
class CSR:
    """An undirected graph in CSR form (both directions stored)."""
    n: int
    off: np.ndarray   # int64 [n+1]
    col: np.ndarray   # int32 [nnz], each row ascending
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.off[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.off)


def kronecker(scale: int, edgefactor: int = 16, seed: int | None = None,
              a: float = KRON_A, b: float = KRON_B, c: float = KRON_C) -> CSR:
    """Kronecker graph of 2^scale vertices from edgefactor*2^scale edge draws."""
    if seed is None:
        seed = 1000 + scale
    st = _load().gg_kronecker(scale, edgefactor, seed, a, b, c, _threads())
    off, col = _emit(st)
    return CSR(1 << scale, off, col, f"kron{scale}_ef{edgefactor}_s{seed}")


def erdos_renyi(n: int, pairs: int, seed: int = 3020) -> CSR:
    """Erdos-Renyi graph: `pairs` uniform unordered pairs over n vertices."""
    st = _load().gg_erdos_renyi(n, pairs, seed, _threads())
    off, col = _emit(st)
    return CSR(n, off, col, f"er_n{n}_m{pairs}_s{seed}")


def pick_roots(g: CSR, k: int, seed: int) -> np.ndarray:
    """k distinct roots drawn uniformly from vertices of nonzero degree."""
    out = np.empty(max(k, 0), dtype=np.int32)
    got = _load().gg_pick_roots(g.n, g.off.ctypes.data, seed, k, out.ctypes.data)
    if got < 0:
        raise MemoryError("pick_roots failed")
    return out[:got].copy()


def uniform_u64(seed: int, tag: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _load().gg_uniform_u64(seed, tag, count, out.ctypes.data)
    return out


def uniform01(seed: int, tag: int, count: int) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits of the counter stream."""
    return (uniform_u64(seed, tag, count) >> np.uint64(11)).astype(np.float64) / float(1 << 53)


# ---------------------------------------------------------------------------
# Small structured graphs for tests (pure numpy).
# ---------------------------------------------------------------------------

def from_edges(n: int, edges, keep_self_loops: bool = False, sort_rows: bool = True,
               keep_duplicates: bool = False, name: str = "") -> CSR:
    """Build a symmetric CSR from an undirected edge list [(u, v), ...]."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    src = np.concatenate([e[:, 0], e[:, 1]])
    dst = np.concatenate([e[:, 1], e[:, 0]])
    if keep_self_loops:
        loops = e[:, 0] == e[:, 1]
        # a self-loop is one stored entry, not two
        keep = np.concatenate([np.ones(len(e), bool), ~loops])
        src, dst = src[keep], dst[keep]
    else:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    if not keep_duplicates:
        key = np.unique(src * max(n, 1) + dst)
        src, dst = key // max(n, 1), key % max(n, 1)
    order = np.lexsort((dst, src)) if sort_rows else np.argsort(src, kind="stable")
    src, dst = src[order], dst[order]
    off = np.zeros(n + 1, dtype=np.int64)
    np.add.at(off, src + 1, 1)
    off = np.cumsum(off).astype(np.int64)
    return CSR(n, off, dst.astype(np.int32), name)


def path_graph(n: int) -> CSR:
    return from_edges(n, [(i, i + 1) for i in range(n - 1)], name=f"path{n}")


def cycle_graph(n: int) -> CSR:
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)], name=f"cycle{n}")


def grid_graph(rows: int, cols: int) -> CSR:
    ed = []
    for r in range(rows):
        for c in range(cols):
            v = r * cols + c
            if c + 1 < cols:
                ed.append((v, v + 1))
            if r + 1 < rows:
                ed.append((v, v + cols))
    return from_edges(rows * cols, ed, name=f"grid{rows}x{cols}")


def star_graph(n: int, center: int = 0) -> CSR:
    return from_edges(n, [(center, i) for i in range(n) if i != center], name=f"star{n}")


def complete_graph(n: int) -> CSR:
    return from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)], name=f"K{n}")


def hypercube_graph(dim: int) -> CSR:
    n = 1 << dim
    return from_edges(n, [(v, v ^ (1 << b)) for v in range(n) for b in range(dim)
                          if v < v ^ (1 << b)], name=f"Q{dim}")


def random_graph(n: int, p: float, seed: int) -> CSR:
    """G(n, p) from the counter stream (one draw per unordered pair)."""
    if n < 2:
        return from_edges(n, [], name=f"gnp{n}")
    iu, ju = np.triu_indices(n, 1)
    r = uniform01(seed, 7, len(iu))
    sel = r < p
    return from_edges(n, np.stack([iu[sel], ju[sel]], 1), name=f"gnp{n}_{p}_{seed}")


# ---------------------------------------------------------------------------
# The workloads (graph sizes, seeds, root counts).
# ---------------------------------------------------------------------------

GRAPH_SEED = {s: 1000 + s for s in range(40)}
ROOT_SEED = {s: 2000 + s for s in range(40)}
ER20_SEED = 3020
SERVE_SEED = 4242


def workload_graph(name: str) -> CSR:
    """Named workload graphs: 'kron<S>' (ef 16) or 'er20'."""
    if name == "er20":
        return erdos_renyi(1 << 20, 4 << 20, ER20_SEED)
    if name.startswith("kron"):
        s = int(name[4:])
        # large graphs take minutes: report each generation phase on stderr
        _load().gg_set_verbose(1 if s >= 24 else 0)
        try:
            return kronecker(s, 16, GRAPH_SEED[s])
        finally:
            _load().gg_set_verbose(0)
    raise ValueError(name)


def workload_roots(name: str, g: CSR, k: int) -> np.ndarray:
    if name == "er20":
        return pick_roots(g, k, 2020 + 1000)
    s = int(name[4:])
    return pick_roots(g, k, ROOT_SEED[s])
