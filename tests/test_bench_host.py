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


def test_join_layer_counters_attributes_dispatches_by_launch_order(tmp_path):
    """Two traversals: the first with layer 0 in the initialisation kernel and
    two binned kernels after layer 1, the second with layer 0 in the layer
    kernel.  Dispatches of other kernels, a finisher and the later statistics
    traversals are ignored; counters of a layer sum its kernels."""
    lm = {"workload": "w", "options": {}, "layer_kernel": "bfs_layer_kernel",
          "roots": [{"root": 5, "layer0_kernel": 2, "layer_launches": 2, "num_layers": 3,
                     "layers": [{"layer": d, "dir": "TD", "n_f": 1, "m_f": 1, "us": 1.0, "td_bytes": 10,
                                 "bu_bytes": 20, "work": [0] * 6} for d in range(3)]},
                    {"root": 7, "layer0_kernel": 0, "layer_launches": 2, "num_layers": 2,
                     "layers": [{"layer": d, "dir": "BU", "n_f": 1, "m_f": 1, "us": 1.0, "td_bytes": 10,
                                 "bu_bytes": 20, "work": [0] * 6} for d in range(2)]}]}
    mp = tmp_path / "map.json"
    mp.write_text(json.dumps(lm))
    seq = ["__amd_rocclr_fillBufferAligned", "hybfs::bfs_init_root_kernel(hybfs::Params, int)",
           "void hybfs::bfs_layer_kernel<0>(hybfs::Params, int, int)",
           "hybfs::bfs_bin_scan_kernel(hybfs::Params, int)", "hybfs::bfs_bin_scatter_kernel(hybfs::Params, int)",
           "void hybfs::bfs_layer_kernel<0>(hybfs::Params, int, int)", "void hybfs::bfs_finish_kernel<0>(hybfs::Params)",
           "hybfs::bfs_init_kernel(hybfs::Params)", "void hybfs::bfs_layer_kernel<0>(hybfs::Params, int, int)",
           "void hybfs::bfs_layer_kernel<0>(hybfs::Params, int, int)", "void hybfs::bfs_finish_kernel<0>(hybfs::Params)",
           "hybfs::bfs_init_root_kernel(hybfs::Params, int)", "void hybfs::bfs_layer_kernel<3>(hybfs::Params, int, int)"]
    lines = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
    for i, name in enumerate(seq):
        lines.append(f'{i + 1},"{name}",FETCH_SIZE,{i + 1}')
        lines.append(f'{i + 1},"{name}",TCC_HIT_sum,3')
        lines.append(f'{i + 1},"{name}",TCC_MISS_sum,1')
    cp = tmp_path / "c.csv"
    cp.write_text("\n".join(lines) + "\n")
    out = bench.join_layer_counters(str(mp), [str(cp)], fetch_factor=2.0)
    r0, r1 = out["roots"]
    assert "fetch_bytes" not in r0["layers"][0]                  # layer 0 ran in the init kernel
    assert r0["layers"][1]["fetch_bytes"] == (3 + 4 + 5) * 1024 * 2.0   # layer kernel + two binned kernels
    assert r0["layers"][2]["fetch_bytes"] == 6 * 1024 * 2.0
    assert r1["layers"][0]["fetch_bytes"] == 9 * 1024 * 2.0
    assert r1["layers"][1]["fetch_bytes"] == 10 * 1024 * 2.0
    assert r0["layers"][1]["l2_hit"] == 0.75


def test_join_batch_counters_takes_the_last_plain_batch(tmp_path):
    """Two plain batches and a profiled one: the dispatches of the second
    (init, seed, push/pull per layer, finisher) are returned in launch order,
    with durations from a kernel trace and counters from a --pmc run; other
    kernels are ignored."""
    bm = {"workload": "w", "k": 64, "batches": [{"layer_launches": 4}, {"layer_launches": 4}],
          "layers": [{"layer": 0, "dir": "TD", "n_f": 1, "m_f": 1, "us": 1.0},
                     {"layer": 1, "dir": "BU", "n_f": 2, "m_f": 2, "us": 1.0}]}
    mp = tmp_path / "bmap.json"
    mp.write_text(json.dumps(bm))
    one = ["hybfs::bfs_batch_init_kernel(hybfs::BParams, hybfs::LanePtrs)",
           "hybfs::bfs_batch_seed_kernel(hybfs::BParams, hybfs::RootSet)",
           "hybfs::bfs_batch_push_kernel(hybfs::BParams, int)", "hybfs::bfs_batch_pull_kernel(hybfs::BParams, int)",
           "hybfs::bfs_batch_push_kernel(hybfs::BParams, int)", "hybfs::bfs_batch_pull_kernel(hybfs::BParams, int)",
           "hybfs::bfs_batch_finish_kernel(hybfs::BParams)"]
    seq = ["__amd_rocclr_fillBufferAligned"] + one + one + one
    tl = ["Dispatch_Id,Kernel_Name,Start_Timestamp,End_Timestamp"]
    cl = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
    for i, name in enumerate(seq):
        tl.append(f'{i + 1},"{name}",{1000 * i},{1000 * i + 500 + i}')
        cl.append(f'{i + 1},"{name}",FETCH_SIZE,{i + 1}')
        cl.append(f'{i + 1},"{name}",TCC_HIT_sum,1')
        cl.append(f'{i + 1},"{name}",TCC_MISS_sum,3')
    tp, cp = tmp_path / "k.csv", tmp_path / "f.csv"
    tp.write_text("\n".join(tl) + "\n")
    cp.write_text("\n".join(cl) + "\n")
    bm2, rows = bench.join_batch_counters(str(mp), [str(tp), str(cp)], fetch_factor=2.0)
    assert [r["kernel"] for r in rows] == [n.split("(")[0].split("::")[-1] for n in one]
    # the second batch's dispatches are seq[8..14], ids 9..15
    assert rows[0]["fetch_bytes"] == 9 * 1024 * 2.0 and rows[-1]["fetch_bytes"] == 15 * 1024 * 2.0
    assert rows[2]["us"] == (500 + 10) / 1e3
    assert rows[3]["l2_hit"] == 0.25 and rows[3]["write_bytes"] is None
