"""Persisted autotune table (bfs_tune_table_get / _put) on the host: round
trips, replacement of an entry with the same key while the others stay,
lines that do not parse or hold invalid options are skipped, a missing file
is BFS_E_NOTFOUND, and the file stays JSON lines a reader can load.  No GPU:
the keys are built by hand."""
from __future__ import annotations

import ctypes
import json
import math
import sys

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



_KEY_FIELDS = {"n": 1 << 20, "nnz": 31399680, "max_degree": 70000, "isolated": 300000, "cus": 256, "mode": 0}
_TUNED = ("alpha", "beta", "probe_k", "td_hub_degree", "grid_blocks", "words_per_wave", "bu_serial_probes",
          "alpha_binned")


def _whole(v):
    """The integer a JSON value stands for, else None (integral floats count)."""
    if isinstance(v, bool) or not isinstance(v, (int, float)):
        return None
    if isinstance(v, float) and (not math.isfinite(v) or v != math.floor(v)):
        return None
    return int(v) if abs(v) <= 9e15 else None


def _valid(o):
    """The ranges the library accepts for the tuned fields."""
    w = o["words_per_wave"]
    return (o["alpha"] > 0 and o["beta"] > 0 and 0 <= o["probe_k"] <= 64 and 256 <= o["td_hub_degree"] <= 1 << 24
            and o["grid_blocks"] >= 0 and 0 <= w <= 64 and w & (w - 1) == 0 and -1 <= o["bu_serial_probes"] <= 1
            and o["alpha_binned"] >= 0)


def _expected(lines):
    """The entry a lookup of the test key returns: the last line that is a JSON
    object with the key, every tuned field a 32-bit integer, a finite best_us
    that does not underflow, and valid options."""
    found = None
    for line in lines:
        try:
            d = json.loads(line)
        except ValueError:
            continue
        if not isinstance(d, dict) or any(_whole(d.get(k)) != v for k, v in _KEY_FIELDS.items()):
            continue
        o = {f: _whole(d.get(f)) for f in _TUNED}
        t = d.get("best_us")
        if any(v is None or not -2**31 <= v < 2**31 for v in o.values()) or not _valid(o):
            continue
        if isinstance(t, bool) or not isinstance(t, (int, float)) or not math.isfinite(t):
            continue
        if t != 0 and abs(t) < sys.float_info.min:
            continue
        found = (o, float(t))
    return found


def test_reader_matches_a_model_of_the_format(lib, tmp_path):
    """Lookups over generated files agree with a Python model of the format
    (any text, JSON objects with arbitrary fields, entries of the key with
    valid and invalid options); a put then replaces every entry of the key."""
    from hypothesis import given, settings, strategies as st

    key = _key()
    p = tmp_path / "t.jsonl"
    anyval = st.one_of(st.integers(-2**40, 2**40), st.floats(allow_nan=True, allow_infinity=True),
                       st.text(max_size=6), st.booleans())
    names = list(_KEY_FIELDS) + list(_TUNED) + ["best_us"]
    noise = st.dictionaries(st.sampled_from(names), anyval, max_size=len(names)).map(json.dumps)
    good = {"alpha": st.integers(1, 80), "beta": st.integers(1, 40), "probe_k": st.integers(0, 64),
            "td_hub_degree": st.sampled_from([256, 1024, 1 << 24]), "grid_blocks": st.integers(0, 2048),
            "words_per_wave": st.sampled_from([0, 1, 2, 4, 8, 16, 32, 64]), "bu_serial_probes": st.integers(-1, 1),
            "alpha_binned": st.integers(0, 12)}
    bad = {"alpha": st.integers(-2, 0), "beta": st.integers(-2, 0), "probe_k": st.sampled_from([-1, 65]),
           "td_hub_degree": st.sampled_from([255, (1 << 24) + 1]), "grid_blocks": st.just(-1),
           "words_per_wave": st.sampled_from([-1, 3, 12, 65, 128]), "bu_serial_probes": st.sampled_from([-2, 2]),
           "alpha_binned": st.just(-1)}

    @st.composite
    def entry(draw):
        d = dict(_KEY_FIELDS)
        if draw(st.integers(0, 5)) == 0:                 # another key, or a key field that is not a whole number
            d[draw(st.sampled_from(list(_KEY_FIELDS)))] = draw(st.one_of(st.integers(0, 3), st.floats()))
        broken = draw(st.sampled_from(_TUNED)) if draw(st.booleans()) else None
        for f in _TUNED:
            v = draw((bad if f == broken else good)[f])
            d[f] = float(v) if draw(st.integers(0, 9)) == 0 else v
        d["best_us"] = draw(st.one_of(st.floats(0, 1e4), st.floats(allow_nan=True, allow_infinity=True)))
        if draw(st.integers(0, 9)) == 0:
            del d[draw(st.sampled_from(sorted(d)))]
        return json.dumps(d)

    line = st.one_of(st.text(max_size=80), noise, entry())

    @settings(max_examples=400, deadline=None)
    @given(st.lists(line, max_size=6), st.integers(1, 64), st.sampled_from([0, 1, 2, 4, 8, 16, 32, 64]))
    def run(lines, alpha, wpw):
        p.write_text("\n".join(lines) + "\n")
        rc, o, t = _get(lib, p, key)
        want = _expected(lines)
        if want is None:
            assert rc == hybfs.BFS_E_NOTFOUND
        else:
            assert rc == hybfs.BFS_OK
            assert {f: getattr(o, f) for f in _TUNED} == want[0] and t == want[1]
        assert _put(lib, p, key, 3.0, alpha=alpha, words_per_wave=wpw) == hybfs.BFS_OK
        rc, o, t = _get(lib, p, key)
        assert rc == hybfs.BFS_OK and (o.alpha, o.words_per_wave, t) == (alpha, wpw, 3.0)
        assert _expected(p.read_text().splitlines())[0]["alpha"] == alpha

    run()


_WRITER = r"""
import sys
from paper_1704_02259_amd import hybfs
import ctypes
lib = hybfs.load()
path, first, count = sys.argv[1], int(sys.argv[2]), int(sys.argv[3])
for i in range(first, first + count):
    k = hybfs.bfs_tune_key()
    k.n, k.nnz, k.max_degree, k.isolated, k.cus, k.mode = 1000 + i, 16000, 90, 7, 256, 0
    o = hybfs.bfs_options_init(alpha=1 + i % 60)
    rc = lib.bfs_tune_table_put(path.encode(), ctypes.byref(k), ctypes.byref(o), float(i))
    if rc != hybfs.BFS_OK:
        sys.exit(f"put {i}: {rc} {lib.bfs_last_error().decode()}")
"""


def test_puts_from_several_processes_all_survive(lib, tmp_path):
    """Processes that put different keys into one table at the same time
    lose none of them: each put reads the table and renames a rewritten copy
    over it under an exclusive lock on a file beside it."""
    import os
    import subprocess
    import sys

    p = tmp_path / "t.jsonl"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, PYTHONPATH=root + os.pathsep + os.environ.get("PYTHONPATH", ""))
    nproc, per = 4, 40
    procs = [subprocess.Popen([sys.executable, "-c", _WRITER, str(p), str(i * per), str(per)], env=env,
                              stdout=subprocess.PIPE, stderr=subprocess.STDOUT) for i in range(nproc)]
    for pr in procs:
        out, _ = pr.communicate(timeout=240)
        assert pr.returncode == 0, out.decode()[-2000:]
    rows = [json.loads(line) for line in p.read_text().splitlines()]
    assert sorted(r["n"] for r in rows) == [1000 + i for i in range(nproc * per)]
    for i in range(nproc * per):
        k = _key(n=1000 + i, nnz=16000, md=90, iso=7)
        rc, o, t = _get(lib, p, k)
        assert rc == hybfs.BFS_OK and o.alpha == 1 + i % 60 and t == float(i)
    assert not list(tmp_path.glob("*.tmp*"))
