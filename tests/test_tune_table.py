"""Persisted autotune table (bfs_tune_table_get / _put) on the host: round
trips, replacement of an entry with the same key while the others stay,
lines that do not parse or hold invalid options are skipped, a missing file
is BFS_E_NOTFOUND, and the file stays JSON lines a reader can load.  No GPU:
the keys are built by hand."""
from __future__ import annotations

import ctypes
import json

import pytest

from paper_1704_02259_amd import hybfs


@pytest.fixture(scope="module")
def lib():
    return hybfs.load()


def _key(n=1 << 20, nnz=31399680, md=70000, iso=300000, cus=256, mode=0):
    k = hybfs.bfs_tune_key()
    k.n, k.nnz, k.max_degree, k.isolated, k.cus, k.mode = n, nnz, md, iso, cus, mode
    return k


def _get(lib, path, key, **base):
    o = hybfs.bfs_options_init(**base)
    t = ctypes.c_double(-1.0)
    rc = lib.bfs_tune_table_get(str(path).encode(), ctypes.byref(key), ctypes.byref(o), ctypes.byref(t))
    return rc, o, t.value


def _put(lib, path, key, best, **kw):
    o = hybfs.bfs_options_init(**kw)
    return lib.bfs_tune_table_put(str(path).encode(), ctypes.byref(key), ctypes.byref(o), best)


def test_missing_file_and_round_trip(lib, tmp_path):
    p = tmp_path / "t.jsonl"
    assert _get(lib, p, _key())[0] == hybfs.BFS_E_NOTFOUND
    assert _put(lib, p, _key(), 101.5, alpha=48, beta=20, probe_k=16, td_hub_degree=1024, grid_blocks=512,
                words_per_wave=4, bu_serial_probes=1, alpha_binned=6) == hybfs.BFS_OK
    rc, o, t = _get(lib, p, _key(), rule=hybfs.RULES["bu"], first_writer=1)
    assert rc == hybfs.BFS_OK and t == 101.5
    assert (o.alpha, o.beta, o.probe_k, o.td_hub_degree, o.grid_blocks, o.words_per_wave, o.bu_serial_probes,
            o.alpha_binned) == (48, 20, 16, 1024, 512, 4, 1, 6)
    # the fields the table does not tune keep the caller's values
    assert o.rule == hybfs.RULES["bu"] and o.first_writer == 1
    # every other key misses: each key field counts
    for kw in (dict(n=1 << 21), dict(nnz=31399681), dict(md=70001), dict(iso=1), dict(cus=128), dict(mode=1)):
        assert _get(lib, p, _key(**kw))[0] == hybfs.BFS_E_NOTFOUND, kw
    rows = [json.loads(line) for line in p.read_text().splitlines()]
    assert rows == [{"scale": 20, "ef": 15, "n": 1 << 20, "nnz": 31399680, "max_degree": 70000, "isolated": 300000,
                     "cus": 256, "mode": 0, "alpha": 48, "beta": 20, "probe_k": 16, "td_hub_degree": 1024,
                     "grid_blocks": 512, "words_per_wave": 4, "bu_serial_probes": 1, "alpha_binned": 6,
                     "best_us": 101.5}]


def test_replace_keeps_other_entries(lib, tmp_path):
    p = tmp_path / "t.jsonl"
    assert _put(lib, p, _key(mode=0), 10.0, alpha=20) == 0
    assert _put(lib, p, _key(mode=1), 20.0, alpha=2, beta=4) == 0
    assert _put(lib, p, _key(n=1 << 26, nnz=2103857030), 30.0, words_per_wave=4) == 0
    assert _put(lib, p, _key(mode=0), 9.0, alpha=48) == 0          # replaces the first entry
    lines = p.read_text().splitlines()
    assert len(lines) == 3
    rc, o, t = _get(lib, p, _key(mode=0))
    assert rc == 0 and o.alpha == 48 and t == 9.0
    rc, o, t = _get(lib, p, _key(mode=1))
    assert rc == 0 and (o.alpha, o.beta) == (2, 4) and t == 20.0
    rc, o, t = _get(lib, p, _key(n=1 << 26, nnz=2103857030))
    assert rc == 0 and o.words_per_wave == 4 and json.loads(lines[1])["scale"] == 26
    assert not list(tmp_path.glob("*.tmp*"))                        # the temporary was renamed


def test_bad_lines_are_skipped(lib, tmp_path):
    p = tmp_path / "t.jsonl"
    assert _put(lib, p, _key(), 5.0, alpha=30) == 0
    good = p.read_text()
    row = json.loads(good)
    bad_alpha = dict(row, alpha=0)            # alpha must be >= 1: not a valid option set
    missing = {k: v for k, v in row.items() if k != "beta"}
    p.write_text(good + "not json at all\n" + json.dumps(bad_alpha) + "\n" + json.dumps(missing) + "\n{\n")
    rc, o, t = _get(lib, p, _key())
    assert rc == 0 and o.alpha == 30 and t == 5.0                   # the last valid entry counts
    p.write_text(json.dumps(bad_alpha) + "\n")
    assert _get(lib, p, _key())[0] == hybfs.BFS_E_NOTFOUND


def test_invalid_arguments(lib, tmp_path):
    p = tmp_path / "t.jsonl"
    k = _key()
    o = hybfs.bfs_options_init()
    assert lib.bfs_tune_table_get(None, ctypes.byref(k), ctypes.byref(o), None) == hybfs.BFS_E_INVALID
    assert lib.bfs_tune_table_get(str(p).encode(), None, ctypes.byref(o), None) == hybfs.BFS_E_INVALID
    assert lib.bfs_tune_table_put(str(p).encode(), ctypes.byref(k), None, 1.0) == hybfs.BFS_E_INVALID
    assert _put(lib, p, k, 1.0, alpha=0) == hybfs.BFS_E_INVALID       # invalid options are not stored
    assert _put(lib, p, _key(mode=2), 1.0) == hybfs.BFS_E_INVALID
    assert _put(lib, p, k, float("nan")) == hybfs.BFS_E_INVALID
    assert not p.exists()
    assert _put(lib, tmp_path / "no_such_dir" / "t.jsonl", k, 1.0) == hybfs.BFS_E_IO
    assert lib.bfs_tune_key_get(None, 0, ctypes.byref(k)) == hybfs.BFS_E_INVALID
