"""The public header is plain C: it compiles with gcc -std=c99, a C program
links against libhybfs.so and calls the host-only entry points, and every
struct the binding mirrors has the same size and field offsets in C and in
the ctypes definitions (no GPU needed)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INC = os.path.join(ROOT, "include")

# ctypes names that differ from the C field names (Python keywords)
C_NAME = {"async_": "async"}

STRUCTS = ["bfs_options", "bfs_layer_stat", "bfs_stats", "bfs_graph_info", "bfs_serve_config",
           "bfs_serve_report", "bfs_tune_report"]


def _binding():
    from paper_1704_02259_amd import _build, hybfs
    if not os.path.exists(_build.LIB):
        _build.build()
    hybfs.load()
    return hybfs, _build.LIB


def _c_program(hybfs) -> str:
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "hybfs.h"', "int main(void) {"]
    for name in STRUCTS:
        cls = getattr(hybfs, name)
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name}.{field} %zu\\n", offsetof({name}, {C_NAME.get(field, field)}));')
    lines += [
        "  bfs_options o; bfs_options_init(&o);",
        '  printf("defaults %d %d %d %d %d\\n", o.rule, o.alpha, o.beta, o.probe_k, o.td_hub_degree);',
        "  int rc = bfs_run(NULL, 0, NULL, NULL, &o, NULL);",
        '  printf("run_null %d %s\\n", rc, bfs_last_error());',
        "  bfs_serve_config c; bfs_serve_config_init(&c);",
        '  printf("serve_defaults %d %d\\n", c.max_batch, c.streams);',
        "  return 0;", "}"]
    return "\n".join(lines) + "\n"


def test_header_is_c99_and_layouts_match(tmp_path):
    hybfs, lib = _binding()
    src = tmp_path / "abi.c"
    src.write_text(_c_program(hybfs))
    exe = tmp_path / "abi"
    cmd = ["gcc", "-std=c99", "-Wall", "-Werror", "-I", INC, str(src), "-o", str(exe), lib,
           "-Wl,-rpath," + os.path.dirname(lib)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0 and "cannot find" in res.stderr:
        pytest.skip("HIP runtime libraries not linkable here: " + res.stderr[:200])
    assert res.returncode == 0, res.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    got = {}
    for line in out.stdout.splitlines():
        k, *v = line.split(" ", 1)
        got[k] = v[0] if v else ""
    for name in STRUCTS:
        cls = getattr(hybfs, name)
        assert int(got[f"{name}"].split()[1]) == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert int(got[f"{name}.{field}"]) == getattr(cls, field).offset, (name, field)
    assert got["defaults"].split() == ["0", "14", "24", "8", "256"]
    assert got["run_null"].startswith("-1")
    assert got["serve_defaults"].split() == ["64", "4"]
