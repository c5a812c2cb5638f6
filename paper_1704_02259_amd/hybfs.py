"""Python binding of libhybfs (ctypes).  Argument marshalling only: every step
of the traversal runs in the library's HIP kernels.  Names follow the C ABI in
include/hybfs.h.  The binding raises if the compiled library is missing; there
is no fallback path."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhybfs.so")

BFS_OK = 0
BFS_E_INVALID = -1
BFS_E_NOMEM = -2
BFS_E_DEVICE = -3
BFS_E_BUSY = -4
BFS_E_NOTFOUND = -5
BFS_E_TIMEOUT = -6
BFS_E_IO = -7

BFS_GRAPH_DEVICE_INPUT = 1
BFS_GRAPH_ASSUME_VALID = 2
BFS_GRAPH_CHECK_SYMMETRY = 4
BFS_GRAPH_SORT_ROWS = 8

BFS_RULE_EDGES = 0
BFS_RULE_TABLE = 1
BFS_RULE_TOPDOWN = 2
BFS_RULE_BOTTOMUP = 3
RULES = {"edges": 0, "beamer": 0, "table": 1, "td": 2, "bu": 3}


class bfs_options(ctypes.Structure):
    _fields_ = [("rule", ctypes.c_int32), ("alpha", ctypes.c_int32), ("beta", ctypes.c_int32),
                ("probe_k", ctypes.c_int32), ("td_hub_degree", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("words_per_wave", ctypes.c_int32),
                ("layers_per_launch", ctypes.c_int32), ("out_on_device", ctypes.c_int32),
                ("async_", ctypes.c_int32), ("profile_layers", ctypes.c_int32),
                ("graph_launch", ctypes.c_int32), ("td_binned", ctypes.c_int32),
                ("first_writer", ctypes.c_int32), ("bu_serial_probes", ctypes.c_int32),
                ("td_queue", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("td_hub_list", ctypes.c_int32), ("alpha_binned", ctypes.c_int32),
                ("bu_filter", ctypes.c_int32), ("count_work", ctypes.c_int32)]


class bfs_layer_stat(ctypes.Structure):
    _fields_ = [("direction", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("n_f", ctypes.c_int64), ("m_f", ctypes.c_int64), ("m_u", ctypes.c_int64),
                ("v_u", ctypes.c_int64), ("t_us", ctypes.c_double), ("kernel_us", ctypes.c_double),
                ("work", ctypes.c_int64 * 6)]


class bfs_stats(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int32), ("num_layers", ctypes.c_int32),
                ("layers", ctypes.POINTER(bfs_layer_stat)), ("reached", ctypes.c_int64),
                ("reached_degree_sum", ctypes.c_int64), ("device_us", ctypes.c_double),
                ("layer_launches", ctypes.c_int32), ("layer0_kernel", ctypes.c_int32),
                ("layer_kernel_us", ctypes.c_double)]


class bfs_graph_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("isolated", ctypes.c_int64),
                ("max_degree", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("grid_blocks", ctypes.c_int32),
                ("block_threads", ctypes.c_int32), ("slab_k", ctypes.c_int32),
                ("chunk_edges", ctypes.c_int32), ("typical_layers", ctypes.c_int32),
                ("hub_degree", ctypes.c_int32), ("hub_chunks", ctypes.c_int64),
                ("batch_workspace_bytes", ctypes.c_int64),
                ("layer_kernel_wide", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class bfs_serve_config(ctypes.Structure):
    _fields_ = [("memory_budget", ctypes.c_int64), ("max_batch", ctypes.c_int32),
                ("streams", ctypes.c_int32), ("queue_capacity", ctypes.c_int32),
                ("out_on_device", ctypes.c_int32), ("alpha", ctypes.c_int32), ("beta", ctypes.c_int32),
                ("batch_threshold", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class bfs_serve_report(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "completed", "failed", "queued", "running",
                                              "batches", "batched_requests", "admission_waits",
                                              "bytes_in_use", "peak_bytes", "memory_budget")] + \
               [(k, ctypes.c_double) for k in ("p50_us", "p99_us", "mean_us", "max_us", "traversed_edges",
                                               "gteps")] + [("evictions", ctypes.c_int64)]


class bfs_tune_key(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("max_degree", ctypes.c_int64),
                ("isolated", ctypes.c_int64), ("cus", ctypes.c_int32), ("mode", ctypes.c_int32)]


class bfs_tune_report(ctypes.Structure):
    _fields_ = [("trials", ctypes.c_int32), ("rounds", ctypes.c_int32), ("start_us", ctypes.c_double),
                ("best_us", ctypes.c_double)]


OPTION_KNOBS = ("rule", "alpha", "beta", "probe_k", "td_hub_degree", "grid_blocks", "words_per_wave",
                "layers_per_launch", "td_binned", "bu_serial_probes", "td_queue", "td_hub_list", "alpha_binned", "bu_filter")


class HybfsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hybfs error {code}: {msg}")
        self.code = code


_lib = None


def _torch_runtime_first():
    """PyTorch ships its own HIP runtime libraries.  A process that starts the
    library's HIP runtime before torch's finds torch without a GPU afterwards,
    so when torch is importable its GPU runtime is started first (the order
    every caller that allocates through torch uses anyway)."""
    try:
        import torch
    except ImportError:
        return
    torch.cuda.is_available()


def load():
    """Load libhybfs.so.  Raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    _torch_runtime_first()
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, u64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                              ctypes.c_uint64)
    sig = {
        "bfs_last_error": (ctypes.c_char_p, []),
        "bfs_options_init": (None, [ctypes.POINTER(bfs_options)]),
        "bfs_graph_create": (ctypes.c_int, [i64, i64, vp, vp, u32, ctypes.POINTER(vp)]),
        "bfs_graph_destroy": (ctypes.c_int, [vp]),
        "bfs_graph_info_get": (ctypes.c_int, [vp, ctypes.POINTER(bfs_graph_info)]),
        "bfs_run": (ctypes.c_int, [vp, i32, vp, vp, ctypes.POINTER(bfs_options),
                                   ctypes.POINTER(bfs_stats)]),
        "bfs_run_batch": (ctypes.c_int, [vp, vp, i32, vp, vp, ctypes.POINTER(bfs_options),
                                         ctypes.POINTER(bfs_stats)]),
        "bfs_graph_sync": (ctypes.c_int, [vp, vp]),
        "bfs_run_noalloc": (ctypes.c_int, [vp, i32, vp, vp, ctypes.POINTER(bfs_options),
                                           ctypes.POINTER(bfs_stats)]),
        "bfs_tune_key_get": (ctypes.c_int, [vp, i32, ctypes.POINTER(bfs_tune_key)]),
        "bfs_tune_table_get": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(bfs_tune_key),
                                              ctypes.POINTER(bfs_options), ctypes.POINTER(ctypes.c_double)]),
        "bfs_tune_table_put": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(bfs_tune_key),
                                              ctypes.POINTER(bfs_options), ctypes.c_double]),
        "bfs_autotune": (ctypes.c_int, [vp, vp, i32, i32, i32, ctypes.POINTER(bfs_options),
                                        ctypes.POINTER(bfs_tune_report)]),
        "bfs_serve_config_init": (None, [ctypes.POINTER(bfs_serve_config)]),
        "bfs_serve_create": (ctypes.c_int, [ctypes.POINTER(bfs_serve_config), ctypes.POINTER(vp)]),
        "bfs_serve_add_graph": (ctypes.c_int, [vp, vp, ctypes.POINTER(i32)]),
        "bfs_serve_submit": (ctypes.c_int, [vp, i32, i32, vp, vp, ctypes.POINTER(u64)]),
        "bfs_serve_poll": (ctypes.c_int, [vp, u64, ctypes.POINTER(i32)]),
        "bfs_serve_wait": (ctypes.c_int, [vp, u64, i64]),
        "bfs_serve_stats": (ctypes.c_int, [vp, ctypes.POINTER(bfs_serve_report)]),
        "bfs_serve_reset_stats": (ctypes.c_int, [vp]),
        "bfs_serve_destroy": (ctypes.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def bfs_last_error() -> str:
    return (load().bfs_last_error() or b"").decode()


def _check(rc: int):
    if rc != BFS_OK:
        raise HybfsError(rc, bfs_last_error())


def bfs_options_init(**kw) -> bfs_options:
    o = bfs_options()
    load().bfs_options_init(ctypes.byref(o))
    for k, v in kw.items():
        if k == "rule" and isinstance(v, str):
            v = RULES[v]
        if k == "async":
            k = "async_"
        setattr(o, k, v)
    return o


def bfs_graph_create(n: int, nnz: int, row_offsets: int, col_indices: int, flags: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(load().bfs_graph_create(n, nnz, row_offsets, col_indices, flags, ctypes.byref(h)))
    return h.value


def bfs_graph_destroy(g: int):
    _check(load().bfs_graph_destroy(g))


def bfs_graph_info_get(g: int) -> bfs_graph_info:
    info = bfs_graph_info()
    _check(load().bfs_graph_info_get(g, ctypes.byref(info)))
    return info


def bfs_run(g: int, root: int, level_out: int, parent_out: int, opt: bfs_options | None = None,
            stats: bfs_stats | None = None):
    _check(load().bfs_run(g, root, level_out, parent_out,
                          ctypes.byref(opt) if opt is not None else None,
                          ctypes.byref(stats) if stats is not None else None))


def bfs_run_noalloc(g: int, root: int, level_out: int, parent_out: int, opt: bfs_options | None = None,
                    stats: bfs_stats | None = None):
    _check(load().bfs_run_noalloc(g, root, level_out, parent_out,
                                  ctypes.byref(opt) if opt is not None else None,
                                  ctypes.byref(stats) if stats is not None else None))


def bfs_run_batch(g: int, roots: int, k: int, level_out: int, parent_out: int,
                  opt: bfs_options | None = None, stats: bfs_stats | None = None):
    _check(load().bfs_run_batch(g, roots, k, level_out, parent_out,
                                ctypes.byref(opt) if opt is not None else None,
                                ctypes.byref(stats) if stats is not None else None))


def bfs_graph_sync(g: int, stream: int | None = None):
    _check(load().bfs_graph_sync(g, stream))


def make_stats(capacity: int = 256) -> tuple[bfs_stats, ctypes.Array]:
    arr = (bfs_layer_stat * max(capacity, 1))()
    st = bfs_stats()
    st.capacity = capacity
    st.layers = ctypes.cast(arr, ctypes.POINTER(bfs_layer_stat))
    return st, arr


def stats_layers(st: bfs_stats, arr) -> list[dict]:
    out = []
    for i in range(min(st.num_layers, st.capacity)):
        r = arr[i]
        out.append({"dir": r.direction, "n_f": r.n_f, "m_f": r.m_f, "m_u": r.m_u, "v_u": r.v_u,
                    "t_us": r.t_us, "kernel_us": r.kernel_us, "work": list(r.work)})
    return out


def _check_out_tensors(torch, level, parent, need: int):
    """Output tensors must be contiguous int32 device tensors of at least
    `need` elements each (checked here because the library only sees
    pointers)."""
    for name, t in (("level", level), ("parent", parent)):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor, got {type(t).__name__}")
        if t.dtype != torch.int32:
            raise TypeError(f"{name} must be int32, got {t.dtype}")
        if not t.is_cuda:
            raise ValueError(f"{name} must be a device tensor")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() < need:
            raise ValueError(f"{name} has {t.numel()} elements, needs {need}")


class Graph:
    """A graph resident on the current GPU (wraps bfs_graph_create)."""

    def __init__(self, off: np.ndarray, col: np.ndarray, flags: int = 0):
        off = np.ascontiguousarray(off, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        self.n = len(off) - 1
        self.nnz = int(off[-1]) if len(off) else 0
        colp = col.ctypes.data if col.size else None
        self.handle = bfs_graph_create(self.n, self.nnz, off.ctypes.data, colp, flags)

    @classmethod
    def from_csr(cls, g, flags: int = 0) -> "Graph":
        return cls(g.off, g.col, flags)

    def info(self) -> bfs_graph_info:
        return bfs_graph_info_get(self.handle)

    def close(self):
        if self.handle:
            bfs_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, root: int, level=None, parent=None, stream=None, stats: bool = False, **kw):
        """Run one BFS.  With torch CUDA tensors for level/parent the outputs stay
        on the device; otherwise numpy arrays are returned."""
        import torch
        dev_out = level is not None
        if level is None:
            level = np.empty(self.n, dtype=np.int32)
            parent = np.empty(self.n, dtype=np.int32)
            lp, pp = level.ctypes.data, parent.ctypes.data
        else:
            _check_out_tensors(torch, level, parent, self.n)
            lp, pp = level.data_ptr(), parent.data_ptr()
            if stream is None:
                stream = torch.cuda.current_stream().cuda_stream
        opt = bfs_options_init(out_on_device=1 if dev_out else 0, stream=stream, **kw)
        st = arr = None
        if stats:
            st, arr = make_stats(4096)
        bfs_run(self.handle, int(root), lp, pp, opt, st)
        if stats:
            return level, parent, {"num_layers": st.num_layers, "reached": st.reached,
                                   "reached_degree_sum": st.reached_degree_sum,
                                   "device_us": st.device_us, "layer_launches": st.layer_launches,
                                   "layer0_kernel": st.layer0_kernel,
                                   "layer_kernel_us": st.layer_kernel_us,
                                   "layers": stats_layers(st, arr)}
        return level, parent

    def run_noalloc(self, root: int, level, parent, stream=None, stats: bool = False, **kw):
        """bfs_run_noalloc: one BFS into device tensors, with the library's
        fixed device scratch instead of a workspace allocation."""
        import torch
        _check_out_tensors(torch, level, parent, self.n)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        opt = bfs_options_init(out_on_device=1, stream=stream, **kw)
        st = arr = None
        if stats:
            st, arr = make_stats(4096)
        bfs_run_noalloc(self.handle, int(root), level.data_ptr(), parent.data_ptr(), opt, st)
        if stats:
            return level, parent, {"num_layers": st.num_layers, "reached": st.reached,
                                   "reached_degree_sum": st.reached_degree_sum,
                                   "layer_launches": st.layer_launches, "layer0_kernel": st.layer0_kernel,
                                   "layers": stats_layers(st, arr)}
        return level, parent

    def autotune(self, roots, mode: str = "single", max_trials: int = 60, stream=None, table=None,
                 write_table=None, **kw):
        """bfs_autotune: returns (options as a dict of keyword arguments for
        run()/run_batch(), report dict).  With `table` (a tune-table path) an
        entry for this graph, device and mode is used instead of tuning
        (report["source"] says which); `write_table` records what tuning
        found."""
        m = 0 if mode == "single" else 1
        opt = bfs_options_init(stream=stream, **kw)
        key = bfs_tune_key()
        _check(load().bfs_tune_key_get(self.handle, m, ctypes.byref(key)))
        if table:
            t = ctypes.c_double(0.0)
            rc = load().bfs_tune_table_get(os.fsencode(table), ctypes.byref(key), ctypes.byref(opt), ctypes.byref(t))
            if rc == BFS_OK:
                return ({k: getattr(opt, k) for k in OPTION_KNOBS},
                        {"trials": 0, "rounds": 0, "start_us": 0.0, "best_us": t.value, "source": "table"})
            if rc != BFS_E_NOTFOUND:
                _check(rc)
        r = np.ascontiguousarray(np.asarray(roots, dtype=np.int32).reshape(-1))
        rep = bfs_tune_report()
        _check(load().bfs_autotune(self.handle, r.ctypes.data, len(r), m, max_trials, ctypes.byref(opt),
                                   ctypes.byref(rep)))
        if write_table:
            _check(load().bfs_tune_table_put(os.fsencode(write_table), ctypes.byref(key), ctypes.byref(opt),
                                             rep.best_us))
        return ({k: getattr(opt, k) for k in OPTION_KNOBS},
                {"trials": rep.trials, "rounds": rep.rounds, "start_us": rep.start_us, "best_us": rep.best_us,
                 "source": "tuned"})

    def run_batch(self, roots, level=None, parent=None, stream=None, stats: bool = False, **kw):
        """Batched BFS from every root in `roots` (bfs_run_batch).  Outputs are
        root-major k x n: torch CUDA tensors stay on the device, otherwise numpy
        arrays of shape (k, n) are returned."""
        import torch
        r = np.ascontiguousarray(np.asarray(roots, dtype=np.int32).reshape(-1))
        k = len(r)
        dev_out = level is not None
        if level is None:
            level = np.empty((k, self.n), dtype=np.int32)
            parent = np.empty((k, self.n), dtype=np.int32)
            lp, pp = level.ctypes.data, parent.ctypes.data
        else:
            _check_out_tensors(torch, level, parent, k * self.n)
            lp, pp = level.data_ptr(), parent.data_ptr()
            if stream is None:
                stream = torch.cuda.current_stream().cuda_stream
        opt = bfs_options_init(out_on_device=1 if dev_out else 0, stream=stream, **kw)
        st = arr = None
        if stats:
            st, arr = make_stats(4096)
        bfs_run_batch(self.handle, r.ctypes.data if k else None, k, lp, pp, opt, st)
        if stats:
            return level, parent, {"num_layers": st.num_layers, "reached": st.reached,
                                   "reached_degree_sum": st.reached_degree_sum,
                                   "device_us": st.device_us, "layer_launches": st.layer_launches,
                                   "layer0_kernel": st.layer0_kernel,
                                   "layer_kernel_us": st.layer_kernel_us,
                                   "layers": stats_layers(st, arr)}
        return level, parent


class Server:
    """BFS serving over resident graphs (wraps bfs_serve_*).  Output buffers
    passed to submit() must stay alive until the query completes."""

    def __init__(self, **cfg):
        c = bfs_serve_config()
        load().bfs_serve_config_init(ctypes.byref(c))
        for k, v in cfg.items():
            setattr(c, k, v)
        self.cfg = c
        h = ctypes.c_void_p()
        _check(load().bfs_serve_create(ctypes.byref(c), ctypes.byref(h)))
        self.handle = h.value
        self._graphs = []

    def add_graph(self, G: Graph) -> int:
        gid = ctypes.c_int32()
        _check(load().bfs_serve_add_graph(self.handle, G.handle, ctypes.byref(gid)))
        self._graphs.append(G)
        return gid.value

    def submit(self, graph_id: int, root: int, level_ptr: int, parent_ptr: int) -> int:
        t = ctypes.c_uint64()
        _check(load().bfs_serve_submit(self.handle, graph_id, root, level_ptr, parent_ptr, ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int32()
        _check(load().bfs_serve_poll(self.handle, ticket, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int, timeout_us: int = -1):
        _check(load().bfs_serve_wait(self.handle, ticket, timeout_us))

    def stats(self) -> dict:
        r = bfs_serve_report()
        _check(load().bfs_serve_stats(self.handle, ctypes.byref(r)))
        return {k: getattr(r, k) for k, _ in r._fields_}

    def reset_stats(self):
        _check(load().bfs_serve_reset_stats(self.handle))

    def close(self):
        if self.handle:
            _check(load().bfs_serve_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
