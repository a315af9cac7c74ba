#!/usr/bin/env python3
"""Throughput of load-balanced CSR SpMV on one MI355X.

One step = one y = A x over the power-law matrix (m = n = 2,000,000, row
lengths min(Zipf(1.8), 200,000), 10 % empty rows, uniform columns, FP32)
with the merge-path schedule (the Sec. 6.2 heuristic's pick) at 256 threads
x 8 items and x split into two column bands over the XCDs, the fastest
candidate of the autotuner here up to timing noise (its own pick is
reported beside): partition, consume, and the band sums plus carries.  `value` is effective HBM GB/s over
algorithmic bytes B = nnz*(s_v + 4) + (m + 1)*4 + n*s_x + m*4 for K
back-to-back steps with the inputs already in HBM.

The same JSON line carries the roofline of the dominant kernel (merge-path
consume, timed by the library's HIP events on the launch stream), the FP64
oracle timed on the host cores, and per-schedule, BF16, forward+backward,
COO/CSC, batched, graph-traversal (SSSP, BFS) and SpGEMM figures on the other workloads
(skip them with --quick).  Accuracy is asserted by the GPU tests, not here:
the oracle runs in this script only as the timed CPU baseline.

    python bench.py [--steps K] [--warmup W] [--quick]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_GBS = 8000.0
METRIC = "SpMV effective HBM GB/s (% of peak) per schedule; fwd+bwd and batched GB/s"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "merge_consume_powerlaw2M_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2301_04792_amd", "csrc", f) for f in ("k_merge.hip", "lb_device.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spmv_bytes(m, n, nnz, sv=4, sx=4, k=1):
    return nnz * (sv + 4) + (m + 1) * 4 + n * sx * k + m * 4 * k


def backward_bytes(m, n, nnz, sv=4, sx=4):
    # values + col_idx read, dvalues written, row_offsets, dy, x read, dx written
    return nnz * (sv + 4) + nnz * 4 + (m + 1) * 4 + m * 4 + n * sx + n * 4


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# ---------------------------------------------------------------- rocprofv3 summaries

def _read_csv(path):
    import csv

    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _find(dirpath, suffix):
    for root, _, files in os.walk(dirpath):
        for fn in sorted(files):
            if fn.endswith(suffix):
                return os.path.join(root, fn)
    return None


def _counter_per_dispatch(rows, kernel_substr, counter):
    """Mean counter value per dispatch of the matching kernel instance that
    was dispatched most often (the timed configuration)."""
    by_name = {}
    for r in rows:
        if kernel_substr in r.get("Kernel_Name", "") and r.get("Counter_Name") == counter:
            by_name.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    if not by_name:
        return None, 0, ""
    name = max(by_name, key=lambda k: len(by_name[k]))
    vals = by_name[name]
    return sum(vals) / len(vals), len(vals), name


def _consume_config(kernel_name):
    """(block, items, x_bands) from a merge_spmv_consume<...> kernel name."""
    import re

    m = re.search(r"merge_spmv_consume<(\d+), (\d+), [^,]+, [^,]+, (\d+)[,>]", kernel_name)
    return (int(m.group(1)), int(m.group(2)), int(m.group(3))) if m else None


def _config_args(cfg):
    return f"--schedule merge_path --block {cfg[0]} --items {cfg[1]} --x-bands {cfg[2]}"


def summarize_profiles(out_dir, prof_root):
    """Write profiles/*.md and the traffic JSON from rocprofv3 CSV output
    (made by the commands recorded in each summary; the merge-path
    configuration in them is the one named by the profiled kernel)."""
    os.makedirs(out_dir, exist_ok=True)
    stats = _find(os.path.join(prof_root, "prof_trace"), "kernel_stats.csv")
    if stats:
        rows = _read_csv(stats)
        names = [r["Name"] for r in rows if _consume_config(r["Name"])]
        cfg = _consume_config(names[0]) if names else (256, 8, 1)
        cmd_trace = ("rocprofv3 --kernel-trace --stats --output-format csv -d prof_out/prof_trace -o trace -- "
                     f"python3 bench.py --quick --no-cpu {_config_args(cfg)} --steps 10 --warmup 3")
        lines = ["# Kernel trace: power-law 2M SpMV, merge-path (bench --quick)", "",
                 f"Command: `{cmd_trace}`", "",
                 "| kernel | calls | avg µs | min µs | max µs | % time |", "|---|---|---|---|---|---|"]
        for r in rows[:12]:
            name = r["Name"]
            name = name if len(name) < 110 else name[:107] + "..."
            lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                         f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
        with open(os.path.join(out_dir, "merge_consume_powerlaw2M_kernel_trace.md"), "w") as f:
            f.write("\n".join(lines) + "\n")
    gstats = _find(os.path.join(prof_root, "prof_graph"), "kernel_stats.csv")
    if gstats:
        cmd_graph = ("rocprofv3 --kernel-trace --stats --output-format csv -d prof_out/prof_graph -o graph -- "
                     "python3 bench.py --graph-only --no-cpu")
        rows = _read_csv(gstats)
        lines = ["# Kernel trace: SSSP and BFS on the 1M-vertex power-law graph (bench --graph-only)", "",
                 f"Command: `{cmd_graph}`", "",
                 "Every schedule of the traversal section runs; each call is one init launch plus the",
                 "advance launches of its host batches (launches after the frontier empties exit at once).", "",
                 "| kernel | calls | avg µs | min µs | max µs | % time |", "|---|---|---|---|---|---|"]
        for r in rows[:16]:
            name = r["Name"]
            name = name if len(name) < 110 else name[:107] + "..."
            lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                         f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
        with open(os.path.join(out_dir, "traversal_powerlaw1M_kernel_trace.md"), "w") as f:
            f.write("\n".join(lines) + "\n")
    fetch = _find(os.path.join(prof_root, "prof_fetch"), "counter_collection.csv")
    write = _find(os.path.join(prof_root, "prof_write"), "counter_collection.csv")
    if fetch and write:
        fr, wr = _read_csv(fetch), _read_csv(write)
        kern = "merge_spmv_consume"
        f_k, nf, name_f = _counter_per_dispatch(fr, kern, "FETCH_SIZE")
        w_k, nw, name_w = _counter_per_dispatch(wr, kern, "WRITE_SIZE")
        # calibration: the 256 MiB device copy run by bench.py --pmc-calib (reads and writes 2^28 bytes)
        copy_f = [float(r["Counter_Value"]) for r in fr if r.get("Counter_Name") == "FETCH_SIZE"
                  and "copy" in r.get("Kernel_Name", "").lower()]
        copy_w = [float(r["Counter_Value"]) for r in wr if r.get("Counter_Name") == "WRITE_SIZE"
                  and "copy" in r.get("Kernel_Name", "").lower()]
        if f_k is not None and w_k is not None and copy_f and copy_w and name_f == name_w:
            known = float(1 << 28)
            ff = known / (max(copy_f) * 1024.0)
            fw = known / (max(copy_w) * 1024.0)
            read_b = f_k * 1024.0 * ff
            write_b = w_k * 1024.0 * fw
            name = name_f
            cfg = _consume_config(name) or (None, None, None)
            data = {"kernel": kern, "workload": "powerlaw_m2M_zipf1.8_cap200k_empty10pct",
                    "kernel_source_hash": kernel_source_hash(),
                    "block_size": cfg[0], "items_per_thread": cfg[1], "x_bands": cfg[2],
                    "fetch_kb_per_dispatch": f_k, "write_kb_per_dispatch": w_k, "dispatches": [nf, nw],
                    "copy_calibration": {"known_bytes": known, "fetch_kb": max(copy_f), "write_kb": max(copy_w),
                                         "fetch_factor": ff, "write_factor": fw},
                    "hbm_read_bytes_per_launch": read_b, "hbm_write_bytes_per_launch": write_b,
                    "hbm_bytes_per_launch": read_b + write_b,
                    "commands": [
                        "rocprofv3 --pmc FETCH_SIZE --output-format csv -d prof_out/prof_fetch -o fetch -- "
                        f"python3 bench.py --quick --no-cpu {_config_args(cfg)} --steps 3 --warmup 1 --pmc-calib",
                        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d prof_out/prof_write -o write -- "
                        f"python3 bench.py --quick --no-cpu {_config_args(cfg)} --steps 3 --warmup 1 --pmc-calib"]}
            try:
                import synthetic as S

                A, _ = S.config_c2()
                data["nnz"] = A.nnz
                data["algorithmic_bytes_per_launch"] = spmv_bytes(A.m, A.n, A.nnz)
            except Exception:  # noqa: BLE001
                pass
            with open(TRAFFIC_FILE, "w") as f:
                json.dump(data, f, indent=1)
            lines = ["# HBM traffic of merge_spmv_consume on the power-law 2M matrix (rocprofv3 PMC)", "",
                     *[f"Command: `{c}`" for c in data["commands"]], "",
                     f"kernel: `{name[:120]}`", "",
                     f"- FETCH_SIZE per dispatch: {f_k:.0f} KB; WRITE_SIZE per dispatch: {w_k:.0f} KB ({nf}/{nw} dispatches)",
                     f"- calibration copy (2^28 bytes read and written): FETCH_SIZE {max(copy_f):.0f} KB, "
                     f"WRITE_SIZE {max(copy_w):.0f} KB -> factors {ff:.3f} (read), {fw:.3f} (write)",
                     f"- HBM bytes per launch: read {read_b / 1e6:.1f} MB + write {write_b / 1e6:.1f} MB = "
                     f"{(read_b + write_b) / 1e6:.1f} MB",
                     f"- algorithmic bytes per launch: {data.get('algorithmic_bytes_per_launch', 0) / 1e6:.1f} MB",
                     "",
                     "FETCH_SIZE counts the bytes L2 fetches over the fabric (from the Infinity Cache or HBM).",
                     "On the copy and on the 1 GiB streaming probe it reads about half the known bytes, so the",
                     "scale factor assumes every fetch is counted like those streaming fetches; the consume",
                     "kernel's fetches are dominated by full-line fills for random x gathers, so the scaled",
                     "figure is an upper estimate and the unscaled one a lower estimate."]
            with open(os.path.join(out_dir, "merge_consume_powerlaw2M_pmc_traffic.md"), "w") as f:
                f.write("\n".join(lines) + "\n")
    return 0


def run_graph(lb, S, dev, no_cpu):
    """SSSP and BFS on the 1M-vertex power-law graph under several schedules
    (and the oracle timed on one host core unless no_cpu)."""
    import numpy as np
    import torch

    # ------------------------------------------------------------ graph traversal (1M vertices)
    t0 = time.time()
    G, src = S.config_c4_graph()
    log(f"[bench] graph generated: {G.m} vertices, {G.nnz} edges in {time.time() - t0:.1f}s")
    Gd = lb.CSR.from_host(G, dev)
    wsg = torch.empty(lb.traversal_workspace_size(Gd), dtype=torch.uint8, device=dev)

    def wall_ms(fn, reps):
        """median wall-clock ms of whole calls (each synchronizes: the host reads the frontier size)."""
        out = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            out.append(time.perf_counter() - t)
        return float(np.median(out)) * 1e3

    gres = {"vertices": G.m, "edges": G.nnz, "source": src,
            "note": "ms per whole traversal (host loop included); gteps = graph edges / time"}
    graph_schedules = (("auto", "auto", {}), ("thread_mapped", "thread_mapped", {}),
                       ("group64", "group_mapped", {"group_size": 64, "tiles_per_group": 1}),
                       ("group1024", "group_mapped", {"group_size": 1024, "tiles_per_group": 1}),
                       ("group64x64", "group_mapped", {"group_size": 64, "tiles_per_group": 64}),
                       ("merge_path", "merge_path", {}),
                       ("work_queue1024", "work_queue", {"group_size": 1024}))
    for algo, fn in (("sssp", lb.sssp), ("bfs", lb.bfs)):
        per = {}
        for name, sch, p in graph_schedules:
            _, its = fn(Gd, src, sch, workspace=wsg, **p)
            ms = wall_ms(lambda: fn(Gd, src, sch, workspace=wsg, **p), 3 if name == "thread_mapped" else 7)
            per[name] = {"ms": round(ms, 3), "iterations": its, "gteps": round(G.nnz / (ms * 1e-3) / 1e9, 3)}
        gres[algo] = per
        log(f"[bench] {algo}: {per}")
    if not no_cpu:  # CPU baseline of the traversals: the oracle, timed
        import oracle

        cs = []
        cb = []
        for _ in range(3):
            t = time.perf_counter()
            oracle.sssp(G.row_offsets, G.col_idx, G.values, src)
            cs.append(time.perf_counter() - t)
            t = time.perf_counter()
            oracle.bfs(G.row_offsets, G.col_idx, src)
            cb.append(time.perf_counter() - t)
        gres["cpu_oracle"] = {"sssp_ms": round(float(np.median(cs)) * 1e3, 2),
                              "bfs_ms": round(float(np.median(cb)) * 1e3, 2), "cores": 1,
                              "kind": "oracle (Dijkstra with a binary heap; FIFO BFS)"}
    del Gd, wsg
    return gres


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--items", type=int, default=0, help="merge-path items per thread (0 = default)")
    ap.add_argument("--block", type=int, default=0, help="merge-path block size (0 = default)")
    ap.add_argument("--x-bands", type=int, default=2,
                    help="merge-path column bands of x, 1 or 2 (the headline uses 2: x of 8 MB is twice one XCD's L2)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--schedule", default="merge_path",
                    help="headline schedule: merge_path (default), auto (autotuned), group_mapped, thread_mapped")
    ap.add_argument("--graph", action="store_true",
                    help="time the headline's K steps as one HIP graph replay instead of eager launches")
    ap.add_argument("--pmc-calib", action="store_true",
                    help="also run one 256 MiB device copy (known bytes) to scale rocprofv3 FETCH/WRITE_SIZE")
    ap.add_argument("--graph-only", action="store_true",
                    help="run only the graph traversals (SSSP, BFS) and print their figures")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="write profiles/ summaries from rocprofv3 CSV output under DIR and exit")
    args = ap.parse_args()
    if args.summarize_profiles:
        return summarize_profiles(os.path.join(ROOT, "profiles"), args.summarize_profiles)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(it would give each GPU an equal diagonal range of the merge path).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2301_04792_amd as lb
    import synthetic as S

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.graph_only:
        print(json.dumps({"graph_powerlaw1M": run_graph(lb, S, dev, args.no_cpu)}), flush=True)
        return 0
    stream = torch.cuda.current_stream(dev)
    flush = torch.empty(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB, larger than L2 + MALL

    def timed(fn, steps, warmup):
        """ms per step over `steps` back-to-back calls (events on the launch stream)."""
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    def cold(fn, reps):
        """median ms of single calls, each after a 1 GiB write that evicts L2 and MALL."""
        out = []
        for r in range(reps):
            flush.fill_(float(r))
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            out.append(a.elapsed_time(b))
        return float(np.median(out))

    def graph_timed(fn, out, steps):
        """ms per call of `steps` calls captured once in a HIP graph and
        replayed once (the same kernels without the host's launch gaps); its
        replays are first checked bit-equal to the eager result, with eager
        calls between them.  None if they differ."""
        fn()
        torch.cuda.synchronize()
        expect = out.clone()
        side = torch.cuda.Stream(dev)
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            for _ in range(3):
                fn()
        stream.wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            for _ in range(steps):
                fn()
        for _ in range(2):
            out.zero_()
            graph.replay()
            torch.cuda.synchronize()
            if not torch.equal(out, expect):
                log("[bench] graph replay differs from the eager result: not timed")
                return None
            fn()
            torch.cuda.synchronize()
        a_ev = torch.cuda.Event(enable_timing=True)
        b_ev = torch.cuda.Event(enable_timing=True)
        a_ev.record(stream)
        graph.replay()
        b_ev.record(stream)
        torch.cuda.synchronize()
        return a_ev.elapsed_time(b_ev) / steps

    def kernel_avg_ms(fn, steps, name):
        lb.profile_reset()
        lb.profile_enable(True)
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        lb.profile_enable(False)
        ms, n = lb.profile_read(name)
        lb.profile_reset()
        return ms / max(n, 1), n

    # ------------------------------------------------------------ headline workload
    t0 = time.time()
    A, x = S.config_c2()
    log(f"[bench] power-law 2M generated: nnz={A.nnz} in {time.time() - t0:.1f}s")
    Ad = lb.CSR.from_host(A, dev)
    xd = torch.from_numpy(x).to(dev)
    y = torch.empty(A.m, dtype=torch.float32, device=dev)
    params = {}
    if args.items:
        params["items_per_thread"] = args.items
    if args.block:
        params["block_size"] = args.block
    if args.x_bands and args.schedule == "merge_path":
        params["x_bands"] = args.x_bands
    head = args.schedule
    if head == "auto" and not params:
        lb.autotune_clear()
        t0 = time.time()
        lb.tune(Ad)  # schedule and tile size picked by timing the candidates on this matrix
        log(f"[bench] autotuned in {time.time() - t0:.1f}s")
    elif head == "auto":
        head = "merge_path"
    sched = lb.resolve_schedule(Ad, head, **params)
    ws = torch.empty(max(lb.workspace_size(Ad, head, **params), 1), dtype=torch.uint8, device=dev)
    dominant = {"merge_path": "merge_consume", "group_mapped": "group_mapped",
                "thread_mapped": "thread_mapped"}[sched["schedule"]]

    def step():
        lb.spmv(Ad, xd, head, y=y, workspace=ws, **params)

    B = spmv_bytes(A.m, A.n, A.nnz)
    # bring the GPU's clocks up before the W warm-up steps: about 0.3 s of
    # untimed steps (a cold GPU times the first hundred calls a few % slow)
    t_end = time.time() + 0.3
    while time.time() < t_end:
        for _ in range(20):
            step()
        torch.cuda.synchronize()
    ms_eager = timed(step, args.steps, args.warmup)
    ms, timing = ms_eager, "eager"
    if args.graph:
        ms_g = graph_timed(step, y, args.steps)
        if ms_g is not None:
            ms, timing = ms_g, "hip_graph"
    value = B / (ms * 1e-3) / 1e9
    log(f"[bench] {sched}: {ms * 1e3:.1f} us/step ({timing}; eager {ms_eager * 1e3:.1f}), {value:.0f} GB/s")
    ms_cold = cold(step, 10)
    consume_ms, launches = kernel_avg_ms(step, args.steps, dominant)
    others = {}
    if dominant == "merge_consume":
        others = {n: round(kernel_avg_ms(step, args.steps, n)[0], 5) for n in
                  ("merge_partition",) + (("merge_finish",) if sched["x_bands"] == 2 else ("merge_fixup",))}
    achieved = B / (consume_ms * 1e-3) / 1e9
    log(f"[bench] {dominant} {consume_ms * 1e3:.1f} us ({achieved:.0f} GB/s), others {others}, "
        f"cold call {ms_cold * 1e3:.1f} us")
    if args.pmc_calib:
        src = torch.ones(1 << 26, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)  # reads and writes exactly 256 MiB
        torch.cuda.synchronize()
        del src, dst

    # ceilings measured live: streaming read of 1 GiB, and the x gather alone
    pout = torch.empty(lb._lib.lb_probe_default_grid() * 256, dtype=torch.float32, device=dev)
    lb.probe_stream_read(flush, pout)
    stream_ms, _ = kernel_avg_ms(lambda: lb.probe_stream_read(flush, pout), 5, "probe_stream")
    gather_ms, _ = kernel_avg_ms(lambda: lb.probe_gather(Ad.col_idx, xd, pout), 5, "probe_gather")
    gather2_ms, _ = kernel_avg_ms(lambda: lb.probe_gather(Ad.col_idx, xd, pout, bands=2), 5, "probe_gather")
    ceilings = {"stream_read_gbs": round(flush.numel() * 4 / (stream_ms * 1e-3) / 1e9, 1),
                "gather_only_ms": round(gather_ms, 5),
                "gather_bound_gbs": round(B / (gather_ms * 1e-3) / 1e9, 1),
                "gather_only_2band_ms": round(gather2_ms, 5),
                "gather_bound_2band_gbs": round(B / (gather2_ms * 1e-3) / 1e9, 1),
                "note": "gather_only = sum of x[col_idx[j]] over all nonzeros, with every XCD gathering from "
                        "all of x (1 band) or each XCD from its half (2 bands, as the x_bands = 2 merge path); "
                        "an SpMV kernel that gathers the same way cannot finish faster"}
    log(f"[bench] ceilings: {ceilings}")

    traffic, traffic_cfg = None, None
    if os.path.exists(TRAFFIC_FILE):
        try:
            with open(TRAFFIC_FILE) as f:
                tr = json.load(f)
            same_cfg = (tr.get("block_size"), tr.get("items_per_thread"), tr.get("x_bands")) == \
                (sched["block_size"], sched["items_per_thread"], sched["x_bands"])
            if tr.get("kernel_source_hash") == kernel_source_hash() and tr.get("nnz") == A.nnz \
                    and dominant == "merge_consume" and same_cfg:
                traffic = tr.get("hbm_bytes_per_launch")
                traffic_cfg = {"block_size": tr.get("block_size"), "items_per_thread": tr.get("items_per_thread"),
                               "x_bands": tr.get("x_bands"),
                               "unscaled_bytes": round((tr.get("fetch_kb_per_dispatch", 0) +
                                                        tr.get("write_kb_per_dispatch", 0)) * 1024)}
        except (OSError, ValueError):
            traffic = None

    result = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "timing": timing,
        "eager_ms_per_step": round(ms_eager, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "powerlaw_m2M_zipf1.8_cap200k_empty10pct", "m": A.m, "n": A.n, "nnz": A.nnz,
                   "seed": 2, "schedule": sched["schedule"], "block_size": sched["block_size"],
                   "items_per_thread": sched["items_per_thread"], "x_bands": sched["x_bands"]},
        "pct_of_peak": round(100 * value / PEAK_GBS, 2),
        "gflops": round(2 * A.nnz / (ms * 1e-3) / 1e9, 2),
        "algorithmic_bytes": B,
        "cold_ms_per_call": round(ms_cold, 5),
        "cold_gbs": round(B / (ms_cold * 1e-3) / 1e9, 2),
        "ceilings": ceilings,
        "roofline": {"kernel": dominant, "bound": "hbm", "achieved": round(achieved, 2),
                     "peak": PEAK_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_GBS, 4),
                     "traffic": traffic, "traffic_profiled_config": traffic_cfg,
                     "avg_launch_ms": round(consume_ms, 5), "launches": launches,
                     "algorithmic_bytes_per_launch": B, "other_kernels_ms": others,
                     # the measured ceiling of a kernel that gathers x the same way (ceilings above)
                     "gather_ceiling_gbs": ceilings["gather_bound_2band_gbs" if sched.get("x_bands") == 2
                                                    else "gather_bound_gbs"],
                     "frac_of_gather_ceiling": round(achieved / ceilings["gather_bound_2band_gbs" if
                                                     sched.get("x_bands") == 2 else "gather_bound_gbs"], 4)},
    }

    # ------------------------------------------------------------ CPU oracle baseline
    if not args.no_cpu:
        import oracle

        orc = oracle.default()
        orc.spmv(A.row_offsets, A.col_idx, A.values, x)  # warm-up
        reps, t_all = 0, []
        start = time.time()
        while reps < 5 and time.time() - start < 20:
            t1 = time.perf_counter()
            orc.spmv(A.row_offsets, A.col_idx, A.values, x)
            t_all.append(time.perf_counter() - t1)
            reps += 1
        cpu_s = float(np.median(t_all))
        threads = orc.num_threads()
        orc.set_num_threads(1)  # the same oracle on one core, as context
        t1 = []
        for _ in range(2):
            t_1 = time.perf_counter()
            orc.spmv(A.row_offsets, A.col_idx, A.values, x)
            t1.append(time.perf_counter() - t_1)
        orc.set_num_threads(threads)
        result["cpu_baseline"] = {"value": round(B / cpu_s / 1e9, 3), "unit": "GB/s", "cores": threads,
                                  "kind": "oracle", "ms_per_call": round(cpu_s * 1e3, 2),
                                  "sample": f"full power-law 2M matrix, FP64 oracle SpMV, median of {reps} calls",
                                  "one_core_ms_per_call": round(min(t1) * 1e3, 2)}
        log(f"[bench] cpu oracle: {cpu_s * 1e3:.0f} ms/call on {orc.num_threads()} threads")

    if args.quick:
        print(json.dumps(result), flush=True)
        return 0

    extra_steps = max(3, min(args.steps, 10))

    # ------------------------------------------------------------ per schedule on the same matrix
    per = {}
    for name, p in (("merge_path", {}), ("merge_path", {"block_size": 512, "items_per_thread": 8}),
                    ("merge_path", {"x_bands": 2}), ("merge_path", {"block_size": 512, "items_per_thread": 8, "x_bands": 2}),
                    ("thread_mapped", {}), ("group_mapped", {"group_size": 64}),
                    ("group_mapped", {"group_size": 256}), ("group_mapped", {"group_size": 32, "tiles_per_group": 32}),
                    ("group_mapped", {"group_size": 1024, "tiles_per_group": 1024}),
                    ("work_queue", {"group_size": 1024})):
        wsz = lb.workspace_size(Ad, name, **p)
        w2 = torch.empty(max(wsz, 1), dtype=torch.uint8, device=dev)
        f = (lambda name=name, p=p, w2=w2: lb.spmv(Ad, xd, name, y=y, workspace=w2, **p))
        t = timed(f, 3 if name == "thread_mapped" else extra_steps, 1)
        key = name + ("" if not p else "_" + "_".join(f"{k}{v}" for k, v in p.items()))
        per[key] = {"ms": round(t, 4), "gbs": round(B / (t * 1e-3) / 1e9, 2),
                    "pct_of_peak": round(100 * B / (t * 1e-3) / 1e9 / PEAK_GBS, 2)}
        log(f"[bench] {key}: {t * 1e3:.1f} us")
    lb.autotune_clear()
    pick = lb.tune(Ad)
    wst = torch.empty(max(lb.workspace_size(Ad, "auto"), 1), dtype=torch.uint8, device=dev)
    t = timed(lambda: lb.spmv(Ad, xd, "auto", y=y, workspace=wst), extra_steps, 1)
    per["auto_tuned"] = {"ms": round(t, 4), "gbs": round(B / (t * 1e-3) / 1e9, 2),
                         "pct_of_peak": round(100 * B / (t * 1e-3) / 1e9 / PEAK_GBS, 2), "schedule": pick}
    lb.autotune_clear()
    del wst
    result["schedules_powerlaw2M"] = per

    # ------------------------------------------------------------ the small uniform matrix (launch-bound)
    A1, x1 = S.config_c1()
    A1d = lb.CSR.from_host(A1, dev)
    x1d = torch.from_numpy(x1).to(dev)
    y1 = torch.empty(A1.m, dtype=torch.float32, device=dev)
    small = {"m": A1.m, "nnz": A1.nnz, "note": "us per call, back to back; accuracy is asserted by the GPU tests"}
    for name, p in (("thread_mapped", {}), ("group_mapped", {"group_size": 64}),
                    ("group_mapped", {"group_size": 64, "tiles_per_group": 64}), ("merge_path", {})):
        ws1 = torch.empty(max(lb.workspace_size(A1d, name, **p), 1), dtype=torch.uint8, device=dev)
        t = timed(lambda name=name, p=p, ws1=ws1: lb.spmv(A1d, x1d, name, y=y1, workspace=ws1, **p), 50, 10)
        key = name + ("" if not p else "_" + "_".join(f"{k}{v}" for k, v in p.items()))
        small[key] = round(t * 1e3, 2)
    result["uniform4096"] = small
    log(f"[bench] uniform 4096: {small}")
    del A1d, x1d, y1

    # ------------------------------------------------------------ BF16 (accuracy is asserted by the GPU tests)
    bf = {}
    Ab = A.with_values(S.to_bf16_bits(A.values))
    xb = S.to_bf16_bits(x)
    Abd = lb.CSR.from_host(Ab, dev)
    xbd = torch.from_numpy(xb.view(np.int16).copy()).view(torch.bfloat16).to(dev)
    wsb = torch.empty(lb.workspace_size(Abd, "merge_path"), dtype=torch.uint8, device=dev)
    t = timed(lambda: lb.spmv(Abd, xbd, "merge_path", y=y, workspace=wsb), extra_steps, 2)
    Bb = spmv_bytes(A.m, A.n, A.nnz, 2, 2)
    bf["powerlaw2M"] = {"ms": round(t, 4), "gbs": round(Bb / (t * 1e-3) / 1e9, 2), "fp32_gbs": round(value, 2)}
    del Abd, xbd
    L, xl = S.config_c3_laplacian()
    Ld = lb.CSR.from_host(L, dev)
    xld = torch.from_numpy(xl).to(dev)
    yl = torch.empty(L.m, dtype=torch.float32, device=dev)
    wsl = torch.empty(lb.workspace_size(Ld, "merge_path"), dtype=torch.uint8, device=dev)
    tl = timed(lambda: lb.spmv(Ld, xld, "merge_path", y=yl, workspace=wsl), extra_steps, 2)
    tlc = cold(lambda: lb.spmv(Ld, xld, "merge_path", y=yl, workspace=wsl), 5)
    Lb = L.with_values(S.to_bf16_bits(L.values))
    xlb = S.to_bf16_bits(xl)
    Lbd = lb.CSR.from_host(Lb, dev)
    xlbd = torch.from_numpy(xlb.view(np.int16).copy()).view(torch.bfloat16).to(dev)
    tlb = timed(lambda: lb.spmv(Lbd, xlbd, "merge_path", y=yl, workspace=wsl), extra_steps, 2)
    tlbc = cold(lambda: lb.spmv(Lbd, xlbd, "merge_path", y=yl, workspace=wsl), 5)
    BL, BLb = spmv_bytes(L.m, L.n, L.nnz), spmv_bytes(L.m, L.n, L.nnz, 2, 2)
    bf["laplacian2048"] = {"nnz": L.nnz, "fp32_ms": round(tl, 4), "fp32_gbs": round(BL / (tl * 1e-3) / 1e9, 2),
                           "fp32_cold_gbs": round(BL / (tlc * 1e-3) / 1e9, 2),
                           "bf16_ms": round(tlb, 4), "bf16_gbs": round(BLb / (tlb * 1e-3) / 1e9, 2),
                           "bf16_cold_gbs": round(BLb / (tlbc * 1e-3) / 1e9, 2), "schedule": "merge_path"}
    # the autotuned pick for each precision (what schedule="auto" runs after lb.tune)
    for key, Md, xmd, Bm in (("fp32", Ld, xld, BL), ("bf16", Lbd, xlbd, BLb)):
        lb.autotune_clear()
        pick = lb.tune(Md)
        wst = torch.empty(max(lb.workspace_size(Md, "auto"), 1), dtype=torch.uint8, device=dev)
        fl = (lambda Md=Md, xmd=xmd, wst=wst: lb.spmv(Md, xmd, "auto", y=yl, workspace=wst))
        tt = timed(fl, extra_steps, 2)
        tg = graph_timed(fl, yl, 20)  # a launch-bound size: the graph removes the gaps between launches
        bf["laplacian2048"][f"{key}_tuned"] = {"ms": round(tt, 4), "gbs": round(Bm / (tt * 1e-3) / 1e9, 2),
                                               "schedule": pick,
                                               "hip_graph_ms": round(tg, 4) if tg is not None else None,
                                               "hip_graph_gbs": round(Bm / (tg * 1e-3) / 1e9, 2) if tg else None}
        del wst
    lb.autotune_clear()
    result["bf16"] = bf
    log(f"[bench] bf16: {bf}")
    del Ld, Lbd, xld, xlbd, yl

    # ------------------------------------------------------------ forward + backward (1M)
    C4, x4 = S.config_c4()
    C4d = lb.CSR.from_host(C4, dev)
    x4d = torch.from_numpy(x4).to(dev)
    dy4 = torch.from_numpy(S.random_vector(44, C4.m)).to(dev)
    y4 = torch.empty(C4.m, dtype=torch.float32, device=dev)
    ws4 = torch.empty(lb.workspace_size(C4d, "merge_path"), dtype=torch.uint8, device=dev)
    tf = timed(lambda: lb.spmv(C4d, x4d, "merge_path", y=y4, workspace=ws4), extra_steps, 2)
    tb = timed(lambda: lb.spmv_backward(C4d, x4d, dy4), extra_steps, 2)
    bw_ms, _ = kernel_avg_ms(lambda: lb.spmv_backward(C4d, x4d, dy4), extra_steps, "backward")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr4 = lb.transpose_pattern(C4d.pattern)  # once per pattern
    torch.cuda.synchronize()
    tbuild = (time.perf_counter() - t0) * 1e3
    tbt = timed(lambda: lb.spmv_backward(C4d, x4d, dy4, transposed=tr4), extra_steps, 2)
    Bf4, Bb4 = spmv_bytes(C4.m, C4.n, C4.nnz), backward_bytes(C4.m, C4.n, C4.nnz)
    result["fwd_bwd_powerlaw1M"] = {"nnz": C4.nnz, "fwd_ms": round(tf, 4), "bwd_ms": round(tb, 4),
                                    "fwd_gbs": round(Bf4 / (tf * 1e-3) / 1e9, 2),
                                    "bwd_gbs": round(Bb4 / (tb * 1e-3) / 1e9, 2),
                                    "bwd_kernel_ms": round(bw_ms, 4),
                                    "bwd_transposed_ms": round(tbt, 4),
                                    "bwd_transposed_gbs": round(Bb4 / (tbt * 1e-3) / 1e9, 2),
                                    "transpose_build_ms": round(tbuild, 3),
                                    "fwd_bwd_transposed_gbs": round((Bf4 + Bb4) / ((tf + tbt) * 1e-3) / 1e9, 2),
                                    "fwd_bwd_gbs": round((Bf4 + Bb4) / ((tf + tb) * 1e-3) / 1e9, 2)}
    log(f"[bench] fwd+bwd: {result['fwd_bwd_powerlaw1M']}")

    # ------------------------------------------------------------ other tile sets (1M): COO and CSC
    fm = {"nnz": C4.nnz, "note": "bytes: CSR nnz*8+(m+1)*4+n*4+m*4; COO nnz*12+n*4+m*4; CSC nnz*8+(n+1)*4+n*4+m*4"}
    Bcoo = C4.nnz * 12 + C4.n * 4 + C4.m * 4
    Bcsc = C4.nnz * 8 + (C4.n + 1) * 4 + C4.n * 4 + C4.m * 4
    fm["csr_merge_path"] = {"ms": round(tf, 4), "gbs": round(Bf4 / (tf * 1e-3) / 1e9, 2)}
    coo4 = lb.COO.from_host(S.to_coo(C4), dev)
    for name, p in (("coo_merge_path", {}), ("coo_thread_mapped", {}), ("coo_group_mapped64", {"group_size": 64})):
        sch = name[4:].replace("64", "")
        wsz = torch.empty(max(1, lb.coo_workspace_size(coo4, sch, **p)), dtype=torch.uint8, device=dev)
        t = timed(lambda: lb.spmv_coo(coo4, x4d, sch, y=y4, workspace=wsz, **p),
                  3 if sch != "merge_path" else extra_steps, 1)
        fm[name] = {"ms": round(t, 4), "gbs": round(Bcoo / (t * 1e-3) / 1e9, 2)}
    del coo4
    csc4 = lb.CSC.from_host(S.to_csc(C4), dev)
    t = timed(lambda: lb.spmv_csc(csc4, x4d, "merge_path", y=y4), extra_steps, 1)
    fm["csc_merge_path"] = {"ms": round(t, 4), "gbs": round(Bcsc / (t * 1e-3) / 1e9, 2)}
    del csc4
    result["formats_powerlaw1M"] = fm
    log(f"[bench] formats: {fm}")
    del C4d, x4d, dy4, y4, ws4

    # ------------------------------------------------------------ batched (512 matrices)
    t0 = time.time()
    BH = S.config_c5()
    log(f"[bench] batched generated: {BH.count} matrices, nnz={BH.nnz} in {time.time() - t0:.1f}s")
    Bd = lb.Batch.from_host(BH, dev)
    bres = {"count": BH.count, "total_rows": BH.total_rows, "nnz": BH.nnz}
    for k in (1, 8):
        Xk = torch.from_numpy(S.random_vector(55, BH.total_cols * k).reshape(-1, k)).to(dev)
        Yk = torch.empty((BH.total_rows, k), dtype=torch.float32, device=dev)
        tuned = lb.tune_batched(Bd, k)
        tk = timed(lambda: lb.batched_spmm(Bd, Xk, "auto", Y=Yk), extra_steps, 2)
        Bk = BH.nnz * 8 + (BH.total_rows + 1) * 4 + BH.total_cols * 4 * k + BH.total_rows * 4 * k
        bres[f"k{k}"] = {"ms": round(tk, 4), "gbs": round(Bk / (tk * 1e-3) / 1e9, 2),
                         "gflops": round(2 * BH.nnz * k / (tk * 1e-3) / 1e9, 2), "schedule": tuned}
        del Xk, Yk
        log(f"[bench] batched k={k}: {bres[f'k{k}']}")
    result["batched_512"] = bres
    del Bd

    result["graph_powerlaw1M"] = run_graph(lb, S, dev, args.no_cpu)

    # ------------------------------------------------------------ SpGEMM
    gm = {"note": "ms per whole C = A A (count, allocation, compute); products = sum over A entries of B row lengths"}
    for name, A in (("laplacian1024_squared", S.laplacian_5pt(3, 1024)[0]),
                    ("powerlaw100k_cap2000_squared", S.powerlaw_csr(80, 100_000, 100_000, 1.8, 2000, 0.1)[0])):
        Ad = lb.CSR.from_host(A, dev)
        prods = int(np.diff(A.row_offsets.astype(np.int64))[A.col_idx].sum())
        C = lb.spgemm(Ad, Ad)
        ms = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            C = lb.spgemm(Ad, Ad)
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1e3)
        t = float(np.median(ms))
        gm[name] = {"nnz_a": A.nnz, "products": prods, "nnz_c": C.nnz, "ms": round(t, 3),
                    "gproducts_per_s": round(prods / (t * 1e-3) / 1e9, 3),
                    "gflops": round(2 * prods / (t * 1e-3) / 1e9, 3)}
        if not args.no_cpu:  # CPU baseline: the oracle, timed
            import oracle

            t0 = time.perf_counter()
            oracle.spgemm(A, A)
            gm[name]["cpu_oracle_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
        del Ad, C
    result["spgemm"] = gm
    log(f"[bench] spgemm: {gm}")

    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
