#!/usr/bin/env python3
"""Benchmark of the single-root hybrid BFS on one MI355X.

A step is one traversal from each of the workload's roots (64 seeded roots of
degree > 0 on a seeded Kronecker graph, SCALE 20 and edgefactor 16 by
default), each a full hybrid BFS writing level and canonical parent arrays
into device buffers.  The graph is resident in HBM before timing starts.

value = harmonic mean over roots of TE_i / t_i (Graph500 TEPS, Section 6.3),
with TE_i the undirected edges in root i's component and t_i the HIP-event
time of its traversal on the stream (timing-only events, no cache flush at
the records), median over the timed steps.

Prints one JSON line.  Also reports the layer kernel's achieved algorithmic
bandwidth against the MI355X HBM peak and the serial CPU oracle's rate on a
bounded sample of the same roots.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "harmonic-mean GTEPS"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class TimingEvent:
    """A HIP event used only for timing, created with hipEventDisableSystemFence:
    a default event writes back and invalidates the caches when it is
    recorded, which adds device time to the window it brackets and cools the
    caches of the work that follows.  Same interface as torch's CUDA events."""
    _hip = None

    def __init__(self):
        import ctypes
        if TimingEvent._hip is None:
            import torch
            # the HIP runtime this process already loaded (torch's copy)
            path = os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so")
            hip = ctypes.CDLL(path if os.path.exists(path) else "libamdhip64.so")
            hip.hipEventCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
            hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
            hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
            hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
            TimingEvent._hip = hip
        self._ctypes = ctypes
        self.ev = ctypes.c_void_p()
        rc = TimingEvent._hip.hipEventCreateWithFlags(ctypes.byref(self.ev), 0x20000000)
        if rc != 0:
            raise RuntimeError(f"hipEventCreateWithFlags failed ({rc})")

    def record(self, stream):
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
        rc = TimingEvent._hip.hipEventRecord(self.ev, self._ctypes.c_void_p(handle))
        if rc != 0:
            raise RuntimeError(f"hipEventRecord failed ({rc})")

    def elapsed_time(self, end) -> float:
        ms = self._ctypes.c_float()
        rc = TimingEvent._hip.hipEventElapsedTime(self._ctypes.byref(ms), self.ev, end.ev)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return ms.value

    def __del__(self):
        try:
            if self.ev and TimingEvent._hip is not None:
                TimingEvent._hip.hipEventDestroy(self.ev)
        except Exception:
            pass


# tuned options of the bench's graphs on MI355X (bfs_tune_table_* format),
# written by `bench.py --retune --write-tune-table`
TUNE_TABLE = os.path.join(ROOT, "paper_1704_02259_amd", "tune_table_mi355x.jsonl")


def kernel_source_hash() -> str:
    """Hash of the code the layer kernel is built from, with comments and
    whitespace removed, so that only a change of code marks the committed
    counter runs as stale."""
    import re
    h = hashlib.sha256()
    for f in ("bfs_kernels.hip", "bfs_device.h", "bfs_wave.h"):
        with open(os.path.join(ROOT, "paper_1704_02259_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update("".join(src.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per layer-kernel launch from committed rocprofv3 counter runs,
    if they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_bfs_layer_kernel_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def batched_leg(torch, hybfs, dev, workload="kron22", k=64, reps=3, table=None, write_table=None):
    """Batched multi-source traversal against single-root runs on the same
    roots: speedup = sum of single-root times / batch time, outputs equal."""
    import inputs
    g = inputs.workload_graph(workload)
    roots = inputs.workload_roots(workload, g, k).astype(np.int32)
    G = hybfs.Graph.from_csr(g, flags=hybfs.BFS_GRAPH_ASSUME_VALID)
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    lv = torch.empty((k, g.n), dtype=torch.int32, device=dev)
    pa = torch.empty((k, g.n), dtype=torch.int32, device=dev)
    blv = torch.empty((k, g.n), dtype=torch.int32, device=dev)
    bpa = torch.empty((k, g.n), dtype=torch.int32, device=dev)
    ev = TimingEvent
    # both sides tuned on the same other roots
    troots = inputs.pick_roots(g, k, inputs.ROOT_SEED[int(workload[4:])] + 500)
    sopt, srep = G.autotune(troots[:16], mode="single", max_trials=24, stream=sp, table=table,
                            write_table=write_table)
    skw = {kk: vv for kk, vv in sopt.items() if kk in ("alpha", "beta", "probe_k", "td_hub_degree", "grid_blocks",
                                                       "words_per_wave", "bu_serial_probes", "alpha_binned")}
    # single-root runs (warm-up pass adapts the launch depth), then timed
    te = []
    for i, r in enumerate(roots):
        _, _, st = G.run(int(r), lv[i], pa[i], stream=sp, stats=True, **skw)
        te.append(st["reached_degree_sum"] / 2.0)
    t_single = np.zeros((reps, k))
    for rep in range(reps):
        for i, r in enumerate(roots):
            a, b = ev(), ev()
            a.record(stream)
            G.run(int(r), lv[i], pa[i], stream=sp, async_=1, **skw)
            b.record(stream)
            stream.synchronize()
            t_single[rep, i] = a.elapsed_time(b)
    bopt, brep = G.autotune(troots, mode="batch", max_trials=24, stream=sp, table=table, write_table=write_table)
    bkw = {kk: vv for kk, vv in bopt.items() if kk in ("alpha", "beta", "grid_blocks", "words_per_wave")}
    G.run_batch(roots, blv, bpa, stream=sp, **bkw)      # warm-up, adapts the batch depth
    # the timed group is one hipGraph launch (captured by the first replay)
    G.run_batch(roots, blv, bpa, stream=sp, graph_launch=1, **bkw)
    t_batch = []
    for rep in range(reps):
        a, b = ev(), ev()
        a.record(stream)
        G.run_batch(roots, blv, bpa, stream=sp, async_=1, graph_launch=1, **bkw)
        b.record(stream)
        stream.synchronize()
        t_batch.append(a.elapsed_time(b))
    equal = bool(torch.equal(lv, blv) and torch.equal(pa, bpa))
    ts = float(np.median(t_single, axis=0).sum())
    tb = float(np.median(t_batch))
    G.close()
    del lv, pa, blv, bpa
    torch.cuda.empty_cache()
    return {"workload": f"kronecker_scale{workload[4:]}_ef16_{k}roots", "roots": k,
            "sum_single_ms": round(ts, 3), "batch_ms": round(tb, 3), "speedup": round(ts / tb, 3),
            "gteps_batch": round(sum(te) / (tb * 1e-3) / 1e9, 2),
            "gteps_single_aggregate": round(sum(te) / (ts * 1e-3) / 1e9, 2), "outputs_equal": equal,
            "batch_options": bkw, "batch_launch": "hipGraph replay", "single_options": skw,
            "tune_trials": brep["trials"], "tune_source": {"single": srep["source"], "batch": brep["source"]}}


SERVE_GRAPHS = ["kron14", "kron16", "kron18", "kron20", "kron22", "er20"]


def serving_leg(torch, hybfs, dev, queries=1000, warm=200, pool=96, streams=4, resident=None):
    """Poisson stream of single-root queries over six resident graphs (graph
    chosen with probability proportional to n, root uniform among degree > 0
    vertices), served with continuous batching.  Saturation throughput comes
    from a burst of all queries at once; then paced streams at 0.5x and 0.9x
    of it report p50/p99 latency and GTEPS."""
    import inputs
    resident = resident or {}
    gs, Gs = [], []
    for name in SERVE_GRAPHS:
        g = resident.get(name) or inputs.workload_graph(name)
        gs.append(g)
        Gs.append(hybfs.Graph.from_csr(g, flags=hybfs.BFS_GRAPH_ASSUME_VALID))
    S = hybfs.Server(streams=streams, max_batch=64)
    ids = [S.add_graph(G) for G in Gs]
    w = np.array([g.n for g in gs], dtype=np.float64)
    w /= w.sum()
    rng = np.random.default_rng(inputs.SERVE_SEED)
    live = [np.nonzero(np.diff(g.off) > 0)[0] for g in gs]

    def draw(m):
        out = []
        for _ in range(m):
            gi = int(rng.choice(len(gs), p=w))
            out.append((gi, int(live[gi][rng.integers(len(live[gi]))])))
        return out

    bufs = [[(torch.empty(g.n, dtype=torch.int32, device=dev), torch.empty(g.n, dtype=torch.int32, device=dev))
             for _ in range(pool)] for g in gs]
    slot_ticket = [[None] * pool for _ in gs]
    slot_root = [[None] * pool for _ in gs]        # the query whose answer the slot holds
    counters = [0] * len(gs)

    def submit(gi, r):
        j = counters[gi] % pool
        counters[gi] += 1
        if slot_ticket[gi][j] is not None:
            S.wait(slot_ticket[gi][j])
        lv, pa = bufs[gi][j]
        t = S.submit(ids[gi], r, lv.data_ptr(), pa.data_ptr())
        slot_ticket[gi][j] = t
        slot_root[gi][j] = r
        return t, j

    def drain():
        for gi in range(len(gs)):
            for j in range(pool):
                if slot_ticket[gi][j] is not None:
                    S.wait(slot_ticket[gi][j])
                    slot_ticket[gi][j] = None

    for gi, r in draw(warm):                       # warm-up: adapts launch depths
        submit(gi, r)
    drain()
    burst = draw(queries)
    S.reset_stats()
    t0 = time.perf_counter()
    for gi, r in burst:
        submit(gi, r)
    drain()
    sat_qps = queries / (time.perf_counter() - t0)
    sat = S.stats()
    out = {"graphs": SERVE_GRAPHS, "streams": streams, "max_batch": 64, "queries": queries,
           "saturation_qps": round(sat_qps, 1), "saturation_gteps": round(sat["gteps"], 2),
           "saturation_p50_us": round(sat["p50_us"], 1), "saturation_p99_us": round(sat["p99_us"], 1),
           "runs": []}
    for frac in (0.5, 0.9):
        lam = frac * sat_qps
        qs = draw(queries)
        gaps = rng.exponential(1.0 / lam, queries)
        S.reset_stats()
        t_next = time.perf_counter()
        for (gi, r), gap in zip(qs, gaps):
            t_next += gap
            while time.perf_counter() < t_next:
                pass
            submit(gi, r)
        drain()
        st = S.stats()
        out["runs"].append({"load": frac, "qps": round(lam, 1), "p50_us": round(st["p50_us"], 1),
                            "p99_us": round(st["p99_us"], 1), "gteps": round(st["gteps"], 2),
                            "mean_batch": round(st["completed"] / max(st["batches"], 1), 2),
                            "completed": st["completed"], "failed": st["failed"]})
    # the answers the last measured run left in the buffers (up to `pool` per
    # graph, most from batched traversals) equal the same queries run alone
    ok, checked = True, 0
    for gi in range(len(gs)):
        l1 = torch.empty(gs[gi].n, dtype=torch.int32, device=dev)
        p1 = torch.empty(gs[gi].n, dtype=torch.int32, device=dev)
        for j in range(pool):
            r = slot_root[gi][j]
            if r is None:
                continue
            Gs[gi].run(r, l1, p1)
            torch.cuda.synchronize()
            lv, pa = bufs[gi][j]
            ok &= bool(torch.equal(lv, l1) and torch.equal(pa, p1))
            checked += 1
    out["served_equal_alone"] = ok
    out["served_checked"] = checked
    S.close()
    for G in Gs:
        G.close()
    del bufs
    torch.cuda.empty_cache()
    return out


def sweep(torch, hybfs, dev, scales=(14, 16, 18, 20, 22), efs=(16, 32, 64), nroots=16):
    """Harmonic-mean GTEPS over a SCALE x edgefactor grid (the shape of the
    paper's Figure 3 workload), single-root traversals with default options,
    16 seeded roots per graph, device outputs."""
    import inputs
    rows = []
    for ef in efs:
        for sc in scales:
            t0 = time.time()
            g = inputs.kronecker(sc, ef, 1000 + sc)
            roots = inputs.pick_roots(g, nroots, 2000 + sc)
            G = hybfs.Graph.from_csr(g, flags=hybfs.BFS_GRAPH_ASSUME_VALID)
            stream = torch.cuda.Stream()
            sp = stream.cuda_stream
            lv = torch.empty(g.n, dtype=torch.int32, device=dev)
            pa = torch.empty(g.n, dtype=torch.int32, device=dev)
            te = []
            for r in roots:
                _, _, st = G.run(int(r), lv, pa, stream=sp, stats=True)
                te.append(st["reached_degree_sum"] / 2.0)
            t = np.zeros((3, len(roots)))
            for rep in range(3):
                for i, r in enumerate(roots):
                    a, b = TimingEvent(), TimingEvent()
                    a.record(stream)
                    G.run(int(r), lv, pa, stream=sp, async_=1)
                    b.record(stream)
                    stream.synchronize()
                    t[rep, i] = a.elapsed_time(b)
            ms = np.median(t, axis=0)
            gt = np.array(te) / (ms * 1e-3) / 1e9
            row = {"scale": sc, "edgefactor": ef, "n": g.n, "nnz": g.nnz, "roots": len(roots),
                   "hm_gteps": round(float(len(gt) / np.sum(1.0 / gt)), 2),
                   "median_root_us": round(float(np.median(ms)) * 1e3, 1)}
            rows.append(row)
            log(f"sweep {row} ({time.time() - t0:.1f}s)")
            G.close()
            del lv, pa
            torch.cuda.empty_cache()
    return rows


def host_output_leg(torch, hybfs, G, g, roots, kw, sp, te, dev_out):
    """The same roots with the outputs in host memory: each synchronous run
    includes the device-to-host copy of its 8n output bytes.  Host wall clock
    per run, pageable numpy arrays and pinned tensors; never the headline."""
    res = {"bytes_per_root": 8 * g.n}
    for kind in ("pageable", "pinned"):
        if kind == "pageable":
            lv = np.empty(g.n, dtype=np.int32)
            pa = np.empty(g.n, dtype=np.int32)
            lp, pp = lv.ctypes.data, pa.ctypes.data
        else:
            lvt = torch.empty(g.n, dtype=torch.int32, pin_memory=True)
            pat = torch.empty(g.n, dtype=torch.int32, pin_memory=True)
            lp, pp = lvt.data_ptr(), pat.data_ptr()
        opt = hybfs.bfs_options_init(out_on_device=0, stream=sp, **kw)
        hybfs.bfs_run(G.handle, int(roots[0]), lp, pp, opt, None)
        ts = []
        for r in roots:
            t0 = time.perf_counter()
            hybfs.bfs_run(G.handle, int(r), lp, pp, opt, None)
            ts.append(time.perf_counter() - t0)
        ts = np.array(ts)
        gt = te / ts / 1e9
        # the last root's host outputs against its device run
        hl, hp = (lv, pa) if kind == "pageable" else (lvt.numpy(), pat.numpy())
        res[kind] = {"gteps_hm": round(float(len(gt) / np.sum(1.0 / gt)), 3),
                     "median_root_us": round(float(np.median(ts)) * 1e6, 1),
                     "copy_gbs_est": None,
                     "equal_device_outputs": bool(np.array_equal(hl, dev_out[0]) and np.array_equal(hp, dev_out[1]))}
    return res


def layer_table(G, g, root, kw, torch, dev):
    """Per-layer breakdown of one traversal (the analogue of the paper's
    Tables 4-7): direction, frontier size and edges, HIP-event time of the
    layer's kernels, the algorithmic bytes of either direction and the
    achieved algorithmic bandwidth of the direction taken."""
    import oracle
    lv = torch.empty(g.n, dtype=torch.int32, device=dev)
    pa = torch.empty(g.n, dtype=torch.int32, device=dev)
    for _ in range(2):
        G.run(int(root), lv, pa, **kw)
    _, _, st = G.run(int(root), lv, pa, stats=True, profile_layers=1, **kw)
    elv, _ = oracle.bfs(g, int(root))
    ab = oracle.algorithmic_bytes(g, elv)
    rows = []
    for d, x in enumerate(st["layers"]):
        td, bu = ab["per_layer"][d] if d < len(ab["per_layer"]) else (0, 0)
        taken = bu if x["dir"] else td
        us = x["kernel_us"]
        rows.append({"layer": d, "dir": "BU" if x["dir"] else "TD", "n_f": x["n_f"], "m_f": x["m_f"],
                     "m_u": x["m_u"], "us": round(us, 1), "td_bytes": td, "bu_bytes": bu,
                     "gbs_taken": round(taken / (us * 1e-6) / 1e9, 1) if us > 0 else None})
    return {"root": int(root), "layers": rows, "total_us": round(st["device_us"], 1)}


def layer_profile(torch, hybfs, dev, workload, nroots, kw, out_path):
    """Per-layer profile of the first nroots roots of a workload, for the
    analogue of the paper's Tables 4-7 with hardware counters.  First one
    plain traversal per root (the dispatches a rocprofv3 counter run of this
    command attributes to layers, in launch order), then per root: HIP-event
    time of each layer's kernels, the layer's work counts (count_work) and
    the oracle's algorithmic bytes of either direction.  Writes the layer map
    (JSON) that join_layer_counters reads."""
    import inputs
    import oracle
    g = inputs.workload_graph(workload)
    roots = [int(r) for r in inputs.workload_roots(workload, g, nroots)]
    G = hybfs.Graph.from_csr(g, flags=hybfs.BFS_GRAPH_ASSUME_VALID)
    lv = torch.empty(g.n, dtype=torch.int32, device=dev)
    pa = torch.empty(g.n, dtype=torch.int32, device=dev)
    launches = []
    for r in roots:
        _, _, st = G.run(r, lv, pa, stats=True, **kw)
        torch.cuda.synchronize()
        launches.append({"root": r, "layer0_kernel": st["layer0_kernel"], "layer_launches": st["layer_launches"],
                         "num_layers": st["num_layers"]})
    info = G.info()
    out = {"workload": workload, "options": kw, "n": g.n, "nnz": g.nnz, "binned_kernels": None, "roots": []}
    for r, la in zip(roots, launches):
        _, _, st = G.run(r, lv, pa, stats=True, profile_layers=1, **kw)
        _, _, sc = G.run(r, lv, pa, stats=True, count_work=1, **kw)
        elv, _ = oracle.bfs(g, r)
        ab = oracle.algorithmic_bytes(g, elv)
        rows = []
        for d, (x, c) in enumerate(zip(st["layers"], sc["layers"])):
            td, bu = ab["per_layer"][d] if d < len(ab["per_layer"]) else (0, 0)
            rows.append({"layer": d, "dir": "BU" if x["dir"] else "TD", "n_f": x["n_f"], "m_f": x["m_f"],
                         "us": round(x["kernel_us"], 1), "td_bytes": td, "bu_bytes": bu, "work": c["work"]})
        out["roots"].append({**la, "layers": rows})
        log(f"layer profile root {r}: {len(rows)} layers")
        del elv
    out["layer_kernel"] = "bfs_layer_kernel_wide" if info.layer_kernel_wide else "bfs_layer_kernel"
    with open(out_path, "w") as f:
        json.dump(out, f)
    G.close()
    return out


def batch_profile(torch, hybfs, dev, workload, nbatches, out_path, k=64):
    """Per-layer profile of the batched traversal of the workload's first k
    roots: nbatches plain batches (direct launches, the dispatches a
    rocprofv3 run of this command attributes to layers in launch order), then
    one batch with per-layer HIP events.  Writes the map join_batch_counters
    reads."""
    import inputs
    g = inputs.workload_graph(workload)
    roots = inputs.workload_roots(workload, g, k).astype(np.int32)
    G = hybfs.Graph.from_csr(g, flags=hybfs.BFS_GRAPH_ASSUME_VALID)
    blv = torch.empty((k, g.n), dtype=torch.int32, device=dev)
    bpa = torch.empty((k, g.n), dtype=torch.int32, device=dev)
    runs = []
    for _ in range(nbatches):
        _, _, st = G.run_batch(roots, blv, bpa, stats=True)
        runs.append({"layer_launches": st["layer_launches"], "num_layers": st["num_layers"],
                     "device_us": round(st["device_us"], 1)})
    _, _, st = G.run_batch(roots, blv, bpa, stats=True, profile_layers=1)
    layers = [{"layer": d, "dir": "BU" if x["dir"] else "TD", "n_f": x["n_f"], "m_f": x["m_f"],
               "us": round(x["kernel_us"], 1)} for d, x in enumerate(st["layers"])]
    out = {"workload": workload, "k": k, "n": g.n, "nnz": g.nnz, "batches": runs, "layers": layers,
           "profiled_device_us": round(st["device_us"], 1)}
    with open(out_path, "w") as f:
        json.dump(out, f)
    G.close()
    return out


def join_batch_counters(map_path, csv_paths, fetch_factor=2.0, write_factor=1.0):
    """Per-dispatch durations (a rocprofv3 --kernel-trace CSV) and counters
    (--pmc CSVs) of the last plain batch batch_profile ran, by launch order:
    a batch starts at its init kernel, then the seed kernel, then one push and
    one pull kernel per enqueued layer, then the finisher and the level pass."""
    import csv
    with open(map_path) as f:
        bm = json.load(f)
    disp = {}
    for p in csv_paths:
        with open(p) as f:
            for r in csv.DictReader(f):
                if "bfs_batch" not in r["Kernel_Name"]:
                    continue
                ent = disp.setdefault(int(r["Dispatch_Id"]), {"name": r["Kernel_Name"].split("(")[0].split("::")[-1]})
                if "Counter_Name" in r:
                    ent[r["Counter_Name"]] = ent.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
                else:
                    ent["ns"] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    groups = []
    for did in sorted(disp):
        if disp[did]["name"] == "bfs_batch_init_kernel":
            groups.append([])
        if groups:
            groups[-1].append(disp[did])
    seq = groups[len(bm["batches"]) - 1]
    rows = []
    for e in seq:
        h, m = e.get("TCC_HIT_sum"), e.get("TCC_MISS_sum")
        rows.append({"kernel": e["name"], "us": e["ns"] / 1e3 if "ns" in e else None,
                     "fetch_bytes": e["FETCH_SIZE"] * 1024 * fetch_factor if "FETCH_SIZE" in e else None,
                     "write_bytes": e["WRITE_SIZE"] * 1024 * write_factor if "WRITE_SIZE" in e else None,
                     "l2_hit": round(h / (h + m), 3) if h is not None and m is not None and h + m else None})
    return bm, rows


def _read_counter_csv(path):
    """Per-dispatch counter values of a rocprofv3 --pmc CSV: {dispatch id:
    (kernel name, {counter: value})}."""
    import csv
    rows = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            did = int(r["Dispatch_Id"])
            name = r["Kernel_Name"]
            ent = rows.setdefault(did, (name, {}))
            ent[1][r["Counter_Name"]] = ent[1].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return rows


def join_layer_counters(map_path, csv_paths, fetch_factor=2.0, write_factor=1.0):
    """Attribute rocprofv3 per-dispatch counters (FETCH_SIZE, WRITE_SIZE,
    TCC_HIT_sum, TCC_MISS_sum; KiB for the first two, scaled by the factors a
    plain device copy gives) to the layers of the traversals layer_profile
    ran first, by launch order: a traversal starts at its initialisation
    kernel; layer i's dispatches are its layer kernel and the binned kernels
    enqueued after it.  Returns the layer map with per-layer bytes and L2 hit
    rates."""
    with open(map_path) as f:
        lm = json.load(f)
    disp = {}
    for p in csv_paths:
        for did, (name, cnt) in _read_counter_csv(p).items():
            ent = disp.setdefault(did, [name, {}])
            ent[1].update(cnt)
    order = sorted(disp)
    trav = []
    for did in order:
        name, cnt = disp[did]
        if "init" in name and ("bfs_init_kernel" in name or "bfs_init_root_kernel" in name):
            trav.append([])
        elif trav and ("bfs_" in name):
            trav[-1].append((name, cnt))
    for ri, root in enumerate(lm["roots"]):
        if ri >= len(trav):
            break
        seq = trav[ri]
        first = 1 if root["layer0_kernel"] else 0
        layer = first - 1
        per = {}
        for name, cnt in seq:
            if "layer_kernel" in name:
                layer += 1
            elif "finish" in name or "root_kernel" in name:
                continue
            acc = per.setdefault(layer, {"FETCH_SIZE": 0.0, "WRITE_SIZE": 0.0, "TCC_HIT_sum": 0.0, "TCC_MISS_sum": 0.0})
            for k in acc:
                acc[k] += cnt.get(k, 0.0)
        for row in root["layers"]:
            c = per.get(row["layer"])
            if c is None:
                continue
            row["fetch_bytes"] = c["FETCH_SIZE"] * 1024 * fetch_factor
            row["write_bytes"] = c["WRITE_SIZE"] * 1024 * write_factor
            hm = c["TCC_HIT_sum"] + c["TCC_MISS_sum"]
            row["l2_hit"] = round(c["TCC_HIT_sum"] / hm, 3) if hm else None
    return lm


def cpu_description() -> dict:
    """Host cores and CPU model of the machine the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"host_cores": os.cpu_count(), "usable_cores": len(os.sched_getaffinity(0)), "cpu_model": model}


def pinned_oracle_times(g, roots, budget_s: float):
    """The serial oracle timed root by root on one core (the calling thread
    pinned to the first core it may use, its previous affinity restored
    afterwards), until budget_s seconds of CPU work are spent (at least one
    root).  Returns the core, per-root seconds, TE and the oracle outputs."""
    import oracle
    allowed = sorted(os.sched_getaffinity(0))
    core = allowed[0]
    os.sched_setaffinity(0, {core})
    ts, tes, outs = [], [], {}
    try:
        for r in roots:
            t0 = time.perf_counter()
            elv, epa = oracle.bfs(g, int(r))
            ts.append(time.perf_counter() - t0)
            tes.append(oracle.traversed_edges(g, elv))
            outs[int(r)] = (elv, epa)
            if sum(ts) >= budget_s:
                break
    finally:
        os.sched_setaffinity(0, set(allowed))
    return core, ts, tes, outs


def oracle_parity(torch, G, g, roots, kw, lv, pa, sp, stream, dev, have, nb):
    """Every root's GPU level/parent (run with the timed options kw) against
    oracle.bfs, compared on the device.  The oracle runs root by root in a
    thread pool; `have` holds outputs already computed.  Also returns the
    exact TE of every root and the algorithmic bytes of the first nb roots."""
    import oracle
    workers = max(1, min(16, len(os.sched_getaffinity(0))))

    def work(ir):
        i, r = ir
        if r in have:
            elv, epa = have[r]
        else:
            elv, epa = oracle.bfs(g, r)
        te_r = oracle.traversed_edges(g, elv)
        ab = oracle.algorithmic_bytes(g, elv) if i < nb else None
        return i, r, te_r, ab, elv, epa

    te = np.zeros(len(roots))
    abytes = [None] * len(roots)
    bad = []
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        for i, r, te_r, ab, elv, epa in ex.map(work, [(i, int(r)) for i, r in enumerate(roots)]):
            te[i] = te_r
            abytes[i] = ab
            G.run(r, lv, pa, stream=sp, **kw)
            stream.synchronize()
            ok = bool(torch.equal(lv, torch.from_numpy(elv).to(dev)) and
                      torch.equal(pa, torch.from_numpy(epa).to(dev)))
            if not ok:
                bad.append(r)
            if g.n >= (1 << 24) or i % 16 == 0:
                log(f"oracle root {i} ({r}): TE {te_r:.0f}, equal {ok}")
            del elv, epa
    return te, abytes, bad, workers


def single_root_leg(torch, hybfs, dev, workload, args, nroots, cpu_budget_s, balg_roots, host_outputs,
                    layer_table_n=0, resident=None):
    """Single-root hybrid BFS from nroots seeded roots of one graph: tuned
    options, timed steps (HIP events per traversal), per-layer kernel times,
    oracle parity of every root, roofline, CPU baseline.  Returns the result
    dict and the generated graph."""
    import inputs
    t0 = time.time()
    g = resident or inputs.workload_graph(workload)
    roots = inputs.workload_roots(workload, g, nroots)
    log(f"graph {workload}: n={g.n} nnz={g.nnz} gen {time.time() - t0:.1f}s, {len(roots)} roots")
    t0 = time.time()
    G = hybfs.Graph.from_csr(g, flags=hybfs.BFS_GRAPH_ASSUME_VALID)
    info = G.info()
    log(f"resident in {time.time() - t0:.1f}s; grid {info.grid_blocks}x{info.block_threads}, "
        f"slab_k {info.slab_k}, hub degree {info.hub_degree}, hub chunks {info.hub_chunks}")

    kw = {}
    if args.alpha:
        kw["alpha"] = args.alpha
    if args.beta:
        kw["beta"] = args.beta
    if args.probe_k >= 0:
        kw["probe_k"] = args.probe_k
    if args.first_writer:
        kw["first_writer"] = 1
    if args.words_per_wave:
        kw["words_per_wave"] = args.words_per_wave

    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    tuning = None
    if not args.no_autotune and not kw:
        # tune on roots other than the measured ones (a different root seed)
        s_ = int(workload[4:]) if workload.startswith("kron") else 20
        troots = inputs.pick_roots(g, 16, inputs.ROOT_SEED.get(s_, 2020) + 500)
        t0 = time.time()
        topt, trep = G.autotune(troots, mode="single", max_trials=args.tune_trials, stream=sp,
                                table=None if args.retune else args.tune_table, write_table=args.write_tune_table)
        kw = {k: v for k, v in topt.items() if k in ("alpha", "beta", "probe_k", "td_hub_degree", "grid_blocks",
                                                       "words_per_wave", "bu_serial_probes", "alpha_binned")}
        tuning = {"options": kw, "source": trep["source"], "trials": trep["trials"], "tune_roots": len(troots),
                  "speedup_on_tune_roots": (round(trep["start_us"] / trep["best_us"], 3)
                                            if trep["source"] == "tuned" else None)}
        log(f"autotune {time.time() - t0:.1f}s: {tuning}")
    lv = torch.empty(g.n, dtype=torch.int32, device=dev)
    pa = torch.empty(g.n, dtype=torch.int32, device=dev)

    # one synchronous run per root first: adapts the launch depth, gives traces
    traces = []
    for r in roots:
        _, _, st = G.run(int(r), lv, pa, stream=sp, stats=True, **kw)
        traces.append(st)
    log("layers per root:", sorted({st["num_layers"] for st in traces}))

    def one_step(evs=None):
        for i, r in enumerate(roots):
            if evs is not None:
                evs[i][0].record(stream)
            G.run(int(r), lv, pa, stream=sp, async_=1, **kw)
            if evs is not None:
                evs[i][1].record(stream)

    for _ in range(args.warmup):
        one_step()
    hybfs.bfs_graph_sync(G.handle, sp)
    torch.cuda.synchronize()

    K = args.steps
    evs = [[[TimingEvent(), TimingEvent()] for _ in roots] for _ in range(K)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(K):
        one_step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    # the timed runs were asynchronous: any device-side failure raises here
    hybfs.bfs_graph_sync(G.handle, sp)
    per_root_ms = np.median(np.array([[a.elapsed_time(b) for a, b in evs[k]] for k in range(K)]), axis=0)
    ms_per_step = wall * 1000.0 / K
    default_ms = None
    if tuning is not None:
        # the same roots with the default options, for comparison
        d_ev = [[TimingEvent(), TimingEvent()] for _ in roots]
        for rep in range(2):
            for i, r in enumerate(roots):
                d_ev[i][0].record(stream)
                G.run(int(r), lv, pa, stream=sp, async_=1)
                d_ev[i][1].record(stream)
            stream.synchronize()
        hybfs.bfs_graph_sync(G.handle, sp)
        default_ms = np.array([a.elapsed_time(b) for a, b in d_ev])
    # per-query latency as a caller sees it: host wall clock of a synchronous
    # run (device outputs, final stream synchronisation included), median of 3
    sync_s = np.zeros((3, len(roots)))
    for rep in range(3):
        for i, r in enumerate(roots):
            t0 = time.perf_counter()
            G.run(int(r), lv, pa, stream=sp, **kw)
            sync_s[rep, i] = time.perf_counter() - t0
    sync_s = np.median(sync_s, axis=0)

    # layer-kernel durations with HIP events around every launch (separate pass)
    prof = []
    for r in roots:
        _, _, st = G.run(int(r), lv, pa, stream=sp, stats=True, profile_layers=1, **kw)
        prof.append(st)

    te = np.array([st["reached_degree_sum"] / 2.0 for st in traces])
    cpu = parity_bad = balg_layers = balg_total = None
    workers = None
    if not args.no_cpu:
        # serial oracle on one core, bounded sample of the same roots
        core, cpu_t, cpu_te, have = pinned_oracle_times(g, roots, cpu_budget_s)
        cpu_rates = np.array(cpu_te) / np.array(cpu_t) / 1e9
        ci = cpu_description()
        cpu = {"value": float(len(cpu_rates) / np.sum(1.0 / cpu_rates)), "unit": "GTEPS", "cores": 1,
               "kind": "oracle", "pinned_core": core, **ci,
               "sample": f"first {len(cpu_t)} of the {len(roots)} roots, serial C oracle (FIFO BFS levels + "
                         f"canonical-parent pass, gcc -O3), one thread pinned to core {core}; "
                         f"{sum(cpu_t):.1f}s of CPU work"}
        log(f"cpu oracle: {cpu['value']:.4f} GTEPS over {len(cpu_t)} roots on core {core} ({ci['cpu_model']})")
        # every root against the oracle with the timed options; exact TE and
        # algorithmic bytes from the oracle
        nb = min(balg_roots, len(roots))
        te, abytes, parity_bad, workers = oracle_parity(torch, G, g, [int(r) for r in roots], kw, lv, pa, sp,
                                                        stream, dev, have, nb)
        del have
        log(f"parity of all {len(roots)} roots with the timed options: {'ok' if not parity_bad else parity_bad}")
        # the layers the layer kernel ran: from layer 0 or 1 (layer 0 of a
        # root of small degree runs in the initialisation or a one-block
        # kernel), one per launch; later layers belong to the finisher
        balg_layers = []
        for ab, st in zip(abytes[:nb], prof[:nb]):
            first = 1 if st["layer0_kernel"] else 0
            pl = ab["per_layer"][first:first + st["layer_launches"]]
            balg_layers.append(sum(min(td, bu) for td, bu in pl))
        balg_total = [ab["bytes"] for ab in abytes[:nb]]

    gteps = te / (per_root_ms * 1e-3) / 1e9
    hm = float(len(gteps) / np.sum(1.0 / gteps))
    if tuning is not None:
        dg = te / (default_ms * 1e-3) / 1e9
        tuning["value_default_options"] = round(float(len(dg) / np.sum(1.0 / dg)), 3)
    agg = float(te.sum() / (ms_per_step * 1e-3) / 1e9)
    sg = te / sync_s / 1e9

    roofline = None
    if balg_layers is not None:
        nb = len(balg_layers)
        launches_b = sum(prof[i]["layer_launches"] for i in range(nb))
        us_b = sum(prof[i]["layer_kernel_us"] for i in range(nb))
        bytes_per_launch = sum(balg_layers) / launches_b
        avg_us = us_b / launches_b
        achieved = bytes_per_launch / (avg_us * 1e-6) / 1e9
        traversal_us = sum(per_root_ms[:nb]) * 1e3
        traffic = measured_traffic(workload)
        roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                    "kernel": ("bfs_layer_kernel_wide" if info.layer_kernel_wide else "bfs_layer_kernel"),
                    "launches": launches_b, "roots_counted": nb,
                    "alg_bytes_per_launch": round(bytes_per_launch, 1), "avg_launch_us": round(avg_us, 3),
                    "traversal_frac": round(sum(balg_total) / (traversal_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 5)}

    host_out = None
    if host_outputs:
        # host output buffers (device-to-host copy included), on the same roots
        G.run(int(roots[-1]), lv, pa, stream=sp, **kw)
        stream.synchronize()
        host_out = host_output_leg(torch, hybfs, G, g, roots, kw, sp, te, (lv.cpu().numpy(), pa.cpu().numpy()))
        for kind in ("pageable", "pinned"):
            # the copy's share of a run: against the device-output median of the timed loop
            extra = host_out[kind]["median_root_us"] - float(np.median(per_root_ms)) * 1e3
            host_out[kind]["copy_gbs_est"] = round(8 * g.n / (extra * 1e-6) / 1e9, 2) if extra > 0 else None
        log("host outputs:", host_out)

    s = int(workload[4:]) if workload.startswith("kron") else None
    res = {
        "value": round(hm, 3),
        "ms_per_step": round(ms_per_step, 4),
        "config": {"workload": (f"kronecker_scale{s}_ef16_{len(roots)}roots_single_root_hybrid_bfs"
                                if s is not None else f"{workload}_{len(roots)}roots"),
                   "n": g.n, "nnz": g.nnz, "roots": len(roots),
                   "graph_seed": inputs.GRAPH_SEED.get(s) if s is not None else inputs.ER20_SEED},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "gteps_aggregate": round(agg, 3),
        "median_root_us": round(float(np.median(per_root_ms)) * 1e3, 2),
        "min_root_gteps": round(float(gteps.min()), 3),
        "sync_wall": {"gteps_hm": round(float(len(sg) / np.sum(1.0 / sg)), 3),
                      "median_root_us": round(float(np.median(sync_s)) * 1e6, 1),
                      "p99_root_us": round(float(np.percentile(sync_s, 99)) * 1e6, 1)},
        "parity_all_roots": None if parity_bad is None else not parity_bad,
        "parity_options": kw,
        "parity_oracle_threads": workers,
        "autotune": tuning,
        "host_outputs": host_out,
    }
    if parity_bad:
        res["parity_failed_roots"] = parity_bad[:16]
    if layer_table_n:
        res["layer_table"] = [layer_table(G, g, r, kw, torch, dev) for r in roots[:layer_table_n]]
        for t in res["layer_table"]:
            log(f"layer table root {t['root']} ({t['total_us']} us):")
            for row in t["layers"]:
                log("  ", row)
    G.close()
    del lv, pa
    torch.cuda.empty_cache()
    return res, g


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="kron20", help="kron<S> (edgefactor 16) or er20")
    ap.add_argument("--roots", type=int, default=64)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="CPU work spent timing the pinned serial oracle (at least one root)")
    ap.add_argument("--balg-roots", type=int, default=64, help="roots whose algorithmic bytes are counted")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle legs (profiling runs)")
    ap.add_argument("--no-s26", action="store_true", help="skip the SCALE-26 block")
    ap.add_argument("--s26-balg-roots", type=int, default=4,
                    help="SCALE-26 roots whose algorithmic bytes are counted (each takes ~30 s of CPU)")
    ap.add_argument("--alpha", type=int, default=0)
    ap.add_argument("--beta", type=int, default=0)
    ap.add_argument("--probe-k", type=int, default=-1)
    ap.add_argument("--words-per-wave", type=int, default=0,
                    help="bottom-up wavefront task size (0: library default); with any option given, "
                         "no tuning pass runs")
    ap.add_argument("--first-writer", action="store_true",
                    help="first-writer top-down parents instead of canonical ones (validated, not compared)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-root leg (SCALE 22)")
    ap.add_argument("--no-autotune", action="store_true", help="time the default options only")
    ap.add_argument("--sweep", action="store_true",
                    help="only the SCALE 14-22 x edgefactor 16/32/64 sweep (one JSON line)")
    ap.add_argument("--layer-table", type=int, default=0,
                    help="also print the per-layer breakdown of this many roots (stderr and JSON)")
    ap.add_argument("--tune-trials", type=int, default=48)
    ap.add_argument("--tune-table", default=TUNE_TABLE,
                    help="persisted autotune table: an entry for a graph, device and mode replaces tuning")
    ap.add_argument("--retune", action="store_true", help="tune even where the table has an entry")
    ap.add_argument("--write-tune-table", default=None, help="record what tuning finds in this table")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-host-out", action="store_true",
                    help="skip the host-output leg (runs that include the device-to-host copy)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (counter calibration)")
    ap.add_argument("--layer-profile", type=int, default=0,
                    help="only the per-layer profile of this many roots of --workload (writes --layer-map)")
    ap.add_argument("--layer-map", default="layer_map.json")
    ap.add_argument("--batch-profile", type=int, default=0,
                    help="N plain batches of the 64 workload roots, then one with per-layer events")
    ap.add_argument("--batch-workload", default="kron22")
    ap.add_argument("--batch-map", default="batch_map.json")
    ap.add_argument("--join-batch-counters", nargs="*", default=None,
                    help="kernel-trace / counter CSVs of a --batch-profile run: per-dispatch table")
    ap.add_argument("--join-counters", nargs="*", default=None,
                    help="host only: join rocprofv3 --pmc CSVs with --layer-map; prints a markdown table")
    args = ap.parse_args()

    if args.join_batch_counters is not None:
        bm, rows = join_batch_counters(args.batch_map, args.join_batch_counters)
        print(f"{bm['workload']}, {bm['k']} roots, dispatches of the last plain batch")
        print("| dispatch | layer | dir | n_f | m_f | µs (trace) | HBM read | HBM write | L2 hit |")
        print("|---|---|---|---|---|---|---|---|---|")
        li = 0
        for i, r in enumerate(rows):
            kind = r["kernel"].replace("bfs_batch_", "").replace("_kernel", "")
            lay = ""
            if kind in ("push", "pull"):
                lay = li
                if kind == "pull":
                    li += 1
            L = bm["layers"][lay] if lay != "" and lay < len(bm["layers"]) else None
            f = lambda x, u: "" if x is None else f"{x / u:.1f}"
            print(f"| {kind} | {lay} | {L['dir'] if L else ''} | {L['n_f'] if L else ''} | {L['m_f'] if L else ''} | "
                  f"{f(r['us'], 1)} | {f(r['fetch_bytes'], 1e6)} MB | {f(r['write_bytes'], 1e6)} MB | "
                  f"{'' if r['l2_hit'] is None else r['l2_hit']} |")
        return
    if args.join_counters is not None:
        lm = join_layer_counters(args.layer_map, args.join_counters)
        print(f"{lm['workload']}, options {lm['options']}, layer kernel {lm['layer_kernel']}")
        print("| root | layer | dir | n_f | m_f | us | alg. bytes (dir taken) | HBM read | HBM write | "
              "hw/alg | L2 hit | work |")
        print("|---|---|---|---|---|---|---|---|---|---|---|---|")
        for root in lm["roots"]:
            for row in root["layers"]:
                alg = row["bu_bytes"] if row["dir"] == "BU" else row["td_bytes"]
                fb, wb = row.get("fetch_bytes"), row.get("write_bytes")
                hw = (fb + wb) if fb is not None else None
                print(f"| {root['root']} | {row['layer']} | {row['dir']} | {row['n_f']} | {row['m_f']} | "
                      f"{row['us']} | {alg / 1e6:.2f} MB | "
                      f"{'' if fb is None else f'{fb / 1e6:.1f} MB'} | {'' if wb is None else f'{wb / 1e6:.1f} MB'} | "
                      f"{'' if hw is None or not alg else f'{hw / alg:.1f}'} | {row.get('l2_hit', '')} | "
                      f"{row['work']} |")
        return

    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4,
                          "launches": 3}))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import inputs
    from paper_1704_02259_amd import _build, hybfs
    if not os.path.exists(_build.LIB) or not os.path.exists(inputs._LIB):
        import __graft_entry__
        __graft_entry__.build()
    hybfs.load()
    if not torch.cuda.is_available():
        sys.exit("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.sweep:
        print(json.dumps({"sweep": sweep(torch, hybfs, dev), "unit": "harmonic-mean GTEPS",
                          "data": "synthetic"}), flush=True)
        return
    if args.batch_profile:
        out = batch_profile(torch, hybfs, dev, args.batch_workload, args.batch_profile, args.batch_map)
        print(json.dumps({"batch_profile": args.batch_workload, "batches": args.batch_profile,
                          "layers": out["layers"], "map": args.batch_map}))
        return
    if args.layer_profile:
        kw = {}
        if args.words_per_wave:
            kw["words_per_wave"] = args.words_per_wave
        if args.alpha:
            kw["alpha"] = args.alpha
        out = layer_profile(torch, hybfs, dev, args.workload, args.layer_profile, kw, args.layer_map)
        print(json.dumps({"layer_profile": args.workload, "roots": len(out["roots"]), "map": args.layer_map}))
        return

    main_leg, g = single_root_leg(torch, hybfs, dev, args.workload, args, args.roots, args.cpu_seconds,
                                  args.balg_roots, not args.no_host_out, args.layer_table)
    out = {
        "metric": METRIC,
        "value": main_leg.pop("value"),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_leg.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": main_leg.pop("config"),
        "roofline": main_leg.pop("roofline"),
        "cpu_baseline": main_leg.pop("cpu_baseline"),
    }
    out.update(main_leg)
    if not args.no_s26 and args.workload == "kron20":
        log("SCALE-26 block (64 roots) ...")
        s26, g26 = single_root_leg(torch, hybfs, dev, "kron26", args, args.roots, args.cpu_seconds,
                                   args.s26_balg_roots, False)
        del g26
        s26 = {"metric": METRIC, "unit": "GTEPS", **s26}
        out["scale26"] = s26
        log("scale26:", {k: s26[k] for k in ("value", "median_root_us", "parity_all_roots", "roofline")})
    if not args.no_batch and args.workload == "kron20":
        log("batched leg (SCALE 22, 64 roots) ...")
        out["batched"] = batched_leg(torch, hybfs, dev, table=None if args.retune else args.tune_table,
                                     write_table=args.write_tune_table)
        log("batched:", out["batched"])
    if not args.no_serve and args.workload == "kron20":
        log("serving leg (6 graphs) ...")
        out["serving"] = serving_leg(torch, hybfs, dev, resident={"kron20": g})
        log("serving:", out["serving"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
