"""The C-ABI library loads without a GPU, exports every symbol its header
declares, and rejects bad arguments on the host before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hybfs.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1704_02259_amd import _build, hybfs
    if not os.path.exists(_build.LIB):
        _build.build()
    return hybfs.load()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(bfs_[a-z_0-9]+)\s*\(",
                                 src, flags=re.M)))


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("bfs_graph_create", "bfs_graph_destroy", "bfs_run", "bfs_run_batch",
                     "bfs_last_error", "bfs_options_init"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_options_defaults(lib):
    from paper_1704_02259_amd import hybfs
    o = hybfs.bfs_options_init()
    assert (o.rule, o.alpha, o.beta, o.probe_k, o.td_hub_degree) == (0, 14, 24, 8, 256)
    assert o.td_binned == 0
    assert (o.grid_blocks, o.words_per_wave, o.layers_per_launch) == (0, 0, 0)
    assert o.out_on_device == 0 and o.async_ == 0 and not o.stream


def _create(lib, n, nnz, off, col, flags=0):
    h = ctypes.c_void_p()
    rc = lib.bfs_graph_create(n, nnz, off.ctypes.data if off is not None else None,
                              col.ctypes.data if col is not None else None, flags, ctypes.byref(h))
    return rc, lib.bfs_last_error().decode()


def test_graph_create_rejects_bad_csr_on_host(lib):
    off = np.array([0, 1, 2], dtype=np.int64)
    col = np.array([1, 0], dtype=np.int32)
    rc, msg = _create(lib, 0, 0, off, col)
    assert rc == -1 and "n =" in msg
    rc, msg = _create(lib, 2, 2, np.array([0, 2, 1], np.int64), col)
    assert rc == -1
    rc, msg = _create(lib, 2, 2, off, np.array([1, 5], np.int32))
    assert rc == -1 and "out of range" in msg
    rc, msg = _create(lib, 2, 3, off, col)
    assert rc == -1 and "nnz" in msg
    # unsorted row without the sort flag
    off3 = np.array([0, 2, 3, 4], np.int64)
    col3 = np.array([2, 1, 0, 0], np.int32)
    rc, msg = _create(lib, 3, 4, off3, col3)
    assert rc == -1 and "sorted" in msg
    # asymmetric graph when symmetry is checked
    off4 = np.array([0, 1, 1], np.int64)
    col4 = np.array([1], np.int32)
    rc, msg = _create(lib, 2, 1, off4, col4, flags=4)
    assert rc == -1 and "reverse" in msg
    # ... also when the structural checks are otherwise skipped
    rc, msg = _create(lib, 2, 1, off4, col4, flags=4 | 2)
    assert rc == -1 and "reverse" in msg
    rc, msg = _create(lib, 2, 2, off, col, flags=1 << 10)
    assert rc == -1 and "flag" in msg


def test_run_rejects_null_graph(lib):
    z = np.zeros(4, np.int32)
    rc = lib.bfs_run(None, 0, z.ctypes.data, z.ctypes.data, None, None)
    assert rc == -1 and "graph" in lib.bfs_last_error().decode()


def test_run_noalloc_rejects_null_graph(lib):
    z = np.zeros(4, np.int32)
    rc = lib.bfs_run_noalloc(None, 0, z.ctypes.data, z.ctypes.data, None, None)
    assert rc == -1 and "graph" in lib.bfs_last_error().decode()


def test_run_batch_rejects_null_graph(lib):
    z = np.zeros(4, np.int32)
    rc = lib.bfs_run_batch(None, z.ctypes.data, 1, z.ctypes.data, z.ctypes.data, None, None)
    assert rc == -1 and "graph" in lib.bfs_last_error().decode()


def test_serve_create_rejects_bad_config(lib):
    from paper_1704_02259_amd import hybfs
    for field, value in (("max_batch", 0), ("max_batch", 65), ("streams", 0), ("streams", 17),
                         ("queue_capacity", 0), ("out_on_device", 2), ("memory_budget", -1),
                         ("batch_threshold", -1), ("batch_threshold", 65)):
        cfg = hybfs.bfs_serve_config()
        lib.bfs_serve_config_init(ctypes.byref(cfg))
        setattr(cfg, field, value)
        h = ctypes.c_void_p()
        assert lib.bfs_serve_create(ctypes.byref(cfg), ctypes.byref(h)) == -1, field
    cfg = hybfs.bfs_serve_config()
    lib.bfs_serve_config_init(ctypes.byref(cfg))
    assert (cfg.max_batch, cfg.streams, cfg.queue_capacity, cfg.out_on_device) == (64, 4, 65536, 1)


def test_serve_calls_reject_null_server(lib):
    z = np.zeros(4, np.int32)
    t = ctypes.c_uint64()
    d = ctypes.c_int32()
    assert lib.bfs_serve_submit(None, 0, 0, z.ctypes.data, z.ctypes.data, ctypes.byref(t)) == -1
    assert lib.bfs_serve_poll(None, 1, ctypes.byref(d)) == -1
    assert lib.bfs_serve_wait(None, 1, 0) == -1
    assert lib.bfs_serve_destroy(None) == -1


def test_autotune_rejects_null_graph(lib):
    from paper_1704_02259_amd import hybfs
    z = np.zeros(4, np.int32)
    o = hybfs.bfs_options_init()
    assert lib.bfs_autotune(None, z.ctypes.data, 1, 0, 10, ctypes.byref(o), None) == -1


def test_binding_raises_without_library(tmp_path, monkeypatch):
    from paper_1704_02259_amd import hybfs
    monkeypatch.setattr(hybfs, "_lib", None)
    monkeypatch.setattr(hybfs, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        hybfs.load()


def test_binding_checks_output_tensors_before_the_call():
    """Wrong dtype, host memory, non-contiguous or short outputs raise in the
    binding (explicit checks, kept under python -O) before any pointer reaches
    the library."""
    import torch
    from paper_1704_02259_amd import hybfs
    good = torch.zeros(8, dtype=torch.int32)
    with pytest.raises(TypeError):
        hybfs._check_out_tensors(torch, np.zeros(8, np.int32), good, 8)
    with pytest.raises(TypeError):
        hybfs._check_out_tensors(torch, torch.zeros(8, dtype=torch.int64), good, 8)
    with pytest.raises(ValueError, match="device"):
        hybfs._check_out_tensors(torch, good, good, 8)
