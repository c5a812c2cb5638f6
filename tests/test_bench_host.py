"""Host-side logic of bench.py (no GPU): the hash that ties committed
counter runs to the layer kernel's code, the lookup of those runs, and the
refusal of more than one GPU."""
from __future__ import annotations

import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

SOURCES = ("bfs_kernels.hip", "bfs_device.h", "bfs_wave.h")


@pytest.fixture()
def tree(tmp_path, monkeypatch):
    """A copy of the kernel sources and profiles that bench.py reads."""
    csrc = tmp_path / "paper_1704_02259_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in SOURCES:
        shutil.copy(os.path.join(ROOT, "paper_1704_02259_amd", "csrc", f), csrc / f)
    shutil.copytree(os.path.join(ROOT, "profiles"), tmp_path / "profiles")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    return tmp_path


def test_hash_ignores_comments_and_whitespace(tree):
    h0 = bench.kernel_source_hash()
    p = tree / "paper_1704_02259_amd" / "csrc" / "bfs_kernels.hip"
    src = p.read_text()
    p.write_text("// a new comment\n/* and a block\n   comment */\n" + src.replace("\n", "\n\n", 5) + "\n   \n")
    assert bench.kernel_source_hash() == h0
    # any change of code is a different hash
    p.write_text(src.replace("kBlock", "kBlock ", 1).replace("return", "return  ", 1) + "\nint x;\n")
    assert bench.kernel_source_hash() != h0


def test_traffic_reported_only_for_matching_code(tree):
    path = tree / "profiles" / "traffic_bfs_layer_kernel_kron20.json"
    t = json.loads(path.read_text())
    t["kernel_source_hash"] = bench.kernel_source_hash()
    path.write_text(json.dumps(t))
    assert bench.measured_traffic("kron20") == t["bytes_per_launch"]
    t["kernel_source_hash"] = "0" * 16
    path.write_text(json.dumps(t))
    assert bench.measured_traffic("kron20") is None
    assert bench.measured_traffic("no_such_workload") is None


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=300)
    line = [l for l in res.stdout.splitlines() if l.startswith("{")][-1]
    out = json.loads(line)
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]
