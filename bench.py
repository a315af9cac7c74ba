#!/usr/bin/env python3
"""Throughput of load-balanced CSR SpMV on one MI355X.

One step = one y = A x over the power-law matrix (m = n = 2,000,000, row
lengths min(Zipf(1.8), 200,000), 10 % empty rows, uniform columns, FP32)
through lb_spmv_planned: a plan built once for the pattern (outside the
timed region; its build time is reported) runs the short rows on the merge
path (128 threads x 8 items, two column bands over the XCDs, the split
precomputed) and the long rows on LDS panels of x, then one finishing pass.
`value` is effective HBM GB/s over algorithmic bytes
B = nnz*(s_v + 4) + (m + 1)*4 + n*s_x + m*4 of the median of the K timed
steps, each run cold: a read of a 1 GiB buffer before it (outside its
events) evicts L2 and the Infinity Cache, the inputs stay in HBM.  The
buffer is written once beforehand, so the lines the eviction leaves behind
are clean: a write right before each step would also charge the step with
writing back up to 256 MB of the buffer's dirty lines (reported beside it
as `cold_write_flush_ms`).  The warm figure (K back-to-back steps) and the
unplanned merge path are reported beside it too.

The same JSON line carries the roofline of the dominant kernel (timed by the
library's HIP events on the launch stream) with every kernel of the call,
the FP64 oracle timed on the host cores (its output also gives the
headline's accuracy, checked outside the timed region), the host CPU, and
per-schedule, BF16, forward+backward, COO/CSC, batched, graph-traversal (SSSP,
BFS) and SpGEMM figures on the other workloads (skip them with --quick).

    python bench.py [--steps K] [--warmup W] [--quick] [--schedule merge_path]
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
# the optional sections and the key of the output line each one fills
SECTION_KEYS = {"schedules": "schedules_powerlaw2M", "uniform": "uniform4096", "bf16": "bf16",
                "fwdbwd": "fwd_bwd_powerlaw1M", "formats": "formats_powerlaw1M", "batched": "batched_512",
                "graph": "graph_powerlaw1M", "spgemm": "spgemm"}
SECTIONS = set(SECTION_KEYS)
METRIC = "SpMV effective HBM GB/s (% of peak) per schedule; fwd+bwd and batched GB/s"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "planned_spmv_powerlaw2M_traffic.json")
kPanelBytes = 163840  # LDS bytes of x per panel block (the library's default panel: 40960 FP32 columns)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2301_04792_amd", "csrc", f)
                  for f in ("k_merge.hip", "k_plan.hip", "lb_device.h", "lb_internal.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spmv_bytes(m, n, nnz, sv=4, sx=4, k=1):
    return nnz * (sv + 4) + (m + 1) * 4 + n * sx * k + m * 4 * k


def backward_bytes(m, n, nnz, sv=4, sx=4):
    # values + col_idx read, dvalues written, row_offsets, dy, x read, dx written
    return nnz * (sv + 4) + nnz * 4 + (m + 1) * 4 + m * 4 + n * sx + n * 4


def host_facts():
    """CPU model and logical CPUs of the machine the bench runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count()}


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


class Records:
    """Measurement records appended to a JSONL file: one line per finished
    section (every configuration, schedule and parameter set it timed, with
    their figures) and one for the headline, each tagged with the kernel
    sources' hash, the device and the host.  With `resume`, a section already
    recorded for the same sources and device is read back instead of measured
    again, so an interrupted sweep continues where it stopped; the headline is
    always measured."""

    def __init__(self, path, resume, device):
        self.path = path
        self.tag = {"kernel_sources": kernel_source_hash(), "device": device}
        self.done = {}
        if path and resume and os.path.exists(path):
            with open(path) as f:
                for line in f:
                    try:
                        r = json.loads(line)
                    except ValueError:  # a line cut short by an interrupted run
                        continue
                    if r.get("section") in SECTION_KEYS and all(r.get(k) == v for k, v in self.tag.items()):
                        self.done[r["section"]] = r["result"]

    def append(self, section, result):
        if not self.path:
            return
        line = {"section": section, **self.tag, "host": host_facts(),
                "time": time.strftime("%Y-%m-%dT%H:%M:%S"), "result": result}
        with open(self.path, "a") as f:
            f.write(json.dumps(line) + "\n")


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


# Profiled runs: tag -> (title, bench.py arguments).  Each kernel trace is
# made by `rocprofv3 --kernel-trace --stats --output-format csv -d
# prof_out/<tag> -o t -- python3 bench.py <arguments>` and summarised into
# profiles/<tag>_kernel_trace.md.
TRACES = {
    "planned_spmv_powerlaw2M": ("planned SpMV on the power-law 2M matrix (the headline)",
                                "--quick --no-cpu --steps 10 --warmup 3"),
    "merge_path_powerlaw2M": ("unplanned two-band merge path on the power-law 2M matrix",
                              "--quick --no-cpu --schedule merge_path --x-bands 2 --steps 10 --warmup 3"),
    "bf16_laplacian_powerlaw2M": ("BF16 on the power-law 2M matrix and the 2048^2 Laplacian (FP32 and BF16), "
                                  "merge path, planned and autotuned", "--only bf16 --no-cpu"),
    "fwd_bwd_powerlaw1M": ("forward, scatter backward and transposed backward on the power-law 1M matrix",
                           "--only fwdbwd --no-cpu"),
    "formats_powerlaw1M": ("COO and CSC on the power-law 1M matrix", "--only formats --no-cpu"),
    "batched512": ("batched SpMM over 512 power-law matrices, k = 1 and k = 8 (autotuned)",
                   "--only batched --no-cpu"),
    "spgemm": ("SpGEMM (Laplacian 1024^2 squared, power-law 100k squared)", "--only spgemm --no-cpu"),
    "uniform4096": ("the 4096^2 uniform matrix (launch-bound): every schedule and the planned call",
                    "--only uniform --no-cpu"),
    "traversal_powerlaw1M": ("SSSP and BFS on the 1M-vertex power-law graph, every schedule",
                             "--graph-only --no-cpu"),
}
# L2-to-memory read requests by size (32, 64 and 128 bytes) and in total:
# their byte sum counts the reads without a scale factor, which checks the
# copy-derived FETCH_SIZE factor on each kernel (FETCH_SIZE counts 128-byte
# requests through TCC_BUBBLE, which does not see them on this chip, so it
# reads half a copy's bytes).
RDREQ_SET = "TCC_EA0_RDREQ_sum TCC_EA0_RDREQ_32B_sum TCC_EA0_RDREQ_64B_sum TCC_EA0_RDREQ_128B_sum"
RDREQ_SIZES = (("TCC_EA0_RDREQ_32B_sum", 32), ("TCC_EA0_RDREQ_64B_sum", 64), ("TCC_EA0_RDREQ_128B_sum", 128))

# Counter passes: tag -> (bench.py arguments, counter sets); each set is one
# `rocprofv3 --pmc <set> --output-format csv -d prof_out/<tag>_<i> -o c --
# python3 bench.py <arguments>` run, summarised into profiles/<tag>_counters.md.
COUNTERS = {
    "planned_spmv_powerlaw2M": ("--quick --no-cpu --steps 3 --warmup 1 --pmc-calib",
                                ["FETCH_SIZE", "WRITE_SIZE",
                                 "SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY "
                                 "SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS SQ_INSTS_VALU",
                                 "TCC_HIT_sum TCC_MISS_sum", "TA_BUSY_avr TA_ADDR_STALLED_BY_TC_CYCLES_sum "
                                 "TCP_PENDING_STALL_CYCLES_sum TCP_TCC_READ_REQ_sum", RDREQ_SET]),
    "fwd_bwd_powerlaw1M": ("--only fwdbwd --no-cpu --steps 3 --pmc-calib",
                           ["FETCH_SIZE", "WRITE_SIZE", "TCC_ATOMIC_sum TCC_EA0_ATOMIC_sum",
                            "SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY", RDREQ_SET]),
    "batched512": ("--only batched --no-cpu --steps 3 --pmc-calib",
                   ["FETCH_SIZE", "WRITE_SIZE", "TCC_HIT_sum TCC_MISS_sum",
                    "SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_ACTIVE_INST_LDS",
                    RDREQ_SET]),
    "bf16_laplacian_powerlaw2M": ("--only bf16 --no-cpu --steps 3 --pmc-calib",
                                  ["FETCH_SIZE", "WRITE_SIZE", "TCC_HIT_sum TCC_MISS_sum",
                                   "SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY "
                                   "SQ_INSTS_VALU SQ_INSTS_LDS SQ_INSTS_SALU", RDREQ_SET]),
}


def _short_name(name, width=100):
    return name if len(name) <= width else name[:width - 3] + "..."


def _copy_calibration(rows):
    """(fetch factor, write factor) from the 256 MiB probe copy run with --pmc-calib, or None."""
    def probe_copy(r):  # the calibration copy: the library's probe_copy_kernel
        return "probe_copy" in r.get("Kernel_Name", "")

    f = [float(r["Counter_Value"]) for r in rows if r.get("Counter_Name") == "FETCH_SIZE" and probe_copy(r)]
    w = [float(r["Counter_Value"]) for r in rows if r.get("Counter_Name") == "WRITE_SIZE" and probe_copy(r)]
    known = float(1 << 28)
    return (known / (max(f) * 1024.0) if f else None, known / (max(w) * 1024.0) if w else None,
            max(f) if f else None, max(w) if w else None)


def _rdreq_bytes(counters):
    """(read bytes, requests not in a size class) from the per-size request
    counts of one kernel, or None without them."""
    if not all(c in counters for c, _ in RDREQ_SIZES) or "TCC_EA0_RDREQ_sum" not in counters:
        return None
    sized = sum(counters[c] for c, _ in RDREQ_SIZES)
    return sum(counters[c] * b for c, b in RDREQ_SIZES), counters["TCC_EA0_RDREQ_sum"] - sized


def summarize_profiles(out_dir, prof_root):
    """Write profiles/*.md (and the headline's traffic JSON) from rocprofv3 CSV
    output under prof_root, made by the commands in TRACES and COUNTERS."""
    import collections

    os.makedirs(out_dir, exist_ok=True)
    for tag, (title, bargs) in TRACES.items():
        stats = _find(os.path.join(prof_root, tag), "kernel_stats.csv")
        if not stats:
            continue
        rows = _read_csv(stats)
        cmd = (f"rocprofv3 --kernel-trace --stats --output-format csv -d prof_out/{tag} -o t -- "
               f"python3 bench.py {bargs}")
        lines = [f"# Kernel trace: {title}", "", f"Command: `{cmd}`", "",
                 "| kernel | calls | avg µs | min µs | max µs | % time |", "|---|---|---|---|---|---|"]
        for r in rows[:24]:
            lines.append(f"| `{_short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                         f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                         f"{float(r['Percentage']):.1f} |")
        with open(os.path.join(out_dir, f"{tag}_kernel_trace.md"), "w") as f:
            f.write("\n".join(lines) + "\n")
    for tag, (bargs, sets) in COUNTERS.items():
        per = collections.defaultdict(dict)  # kernel -> counter -> mean per dispatch
        calls = collections.defaultdict(int)
        cmds, all_rows = [], []
        for i, cset in enumerate(sets):
            path = _find(os.path.join(prof_root, f"{tag}_{i}"), "counter_collection.csv")
            if not path:
                continue
            cmds.append(f"rocprofv3 --pmc {cset} --output-format csv -d prof_out/{tag}_{i} -o c -- "
                        f"python3 bench.py {bargs}")
            rows = _read_csv(path)
            all_rows += rows
            acc = collections.defaultdict(list)
            for r in rows:
                acc[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
            for (k, c), v in acc.items():
                per[k][c] = sum(v) / len(v)
                calls[k] = max(calls[k], len(v))
        if not per:
            continue
        ff, fw, cf, cw = _copy_calibration(all_rows)
        copy_k = [k for k in per if "probe_copy" in k]
        copy_rd = _rdreq_bytes(per[copy_k[0]]) if copy_k else None
        sized = False
        for k in per:
            rb = _rdreq_bytes(per[k])
            if rb:
                per[k]["rdreq_bytes"], per[k]["rdreq_unsized"] = rb
                sized = True
        counters = sorted({c for k in per for c in per[k]})
        lines = [f"# Counters per dispatch: {TRACES.get(tag, (tag,))[0]}", ""] + [f"Command: `{c}`" for c in cmds] + [
            "", "Mean value per dispatch of each kernel (FETCH_SIZE / WRITE_SIZE in KiB; the SQ cycle counters "
                "are in the units rocprofv3 reports, summed over the chip).", ""]
        if ff and fw:
            lines += [f"Copy calibration (a 256 MiB device copy that reads and writes 2^28 bytes): FETCH_SIZE "
                      f"{cf:.0f} KiB, WRITE_SIZE {cw:.0f} KiB, so HBM bytes = FETCH_SIZE x 1024 x {ff:.3f} and "
                      f"WRITE_SIZE x 1024 x {fw:.3f}.", ""]
        if sized:
            lines += ["Read bytes counted by request size: 32 x TCC_EA0_RDREQ_32B + 64 x TCC_EA0_RDREQ_64B + "
                      "128 x TCC_EA0_RDREQ_128B per dispatch (`rdreq_bytes`, no scale factor; "
                      "`rdreq_unsized` = requests outside the three classes)." +
                      (f" On the calibration copy they give {copy_rd[0]:.6g} bytes against the 2^28 = "
                       f"{float(1 << 28):.6g} it reads." if copy_rd else ""), ""]
        lines += ["| kernel | dispatches | " + " | ".join(counters) + " |", "|---|---|" + "---|" * len(counters)]
        for k in sorted(per, key=lambda k: -per[k].get("FETCH_SIZE", 0)):
            if "copy" in k.lower() or "fill" in k.lower():
                continue
            lines.append(f"| `{_short_name(k, 80)}` | {calls[k]} | " +
                         " | ".join(f"{per[k][c]:.4g}" if c in per[k] else "" for c in counters) + " |")
        with open(os.path.join(out_dir, f"{tag}_counters.md"), "w") as f:
            f.write("\n".join(lines) + "\n")
        if tag == "planned_spmv_powerlaw2M" and ff and fw:
            # traffic of the headline's dominant kernel (the short rows' merge-path consume)
            cand = [k for k in per if "merge_spmv_consume" in k and "FETCH_SIZE" in per[k] and "WRITE_SIZE" in per[k]]
            if cand:
                k = max(cand, key=lambda k: calls[k])
                m = _consume_config(k) or (None, None, None)
                read_b, write_b = per[k]["FETCH_SIZE"] * 1024.0 * ff, per[k]["WRITE_SIZE"] * 1024.0 * fw
                # the copy-calibrated FETCH_SIZE, checked against the reads counted by request size
                rd = per[k].get("rdreq_bytes")
                data = {"kernel": "merge_consume", "schedule": "planned", "kernel_name": k,
                        "workload": "powerlaw_m2M_zipf1.8_cap200k_empty10pct",
                        "kernel_source_hash": kernel_source_hash(), "block_size": m[0], "items_per_thread": m[1],
                        "x_bands": m[2], "long_min": None,
                        "fetch_kb_per_dispatch": per[k]["FETCH_SIZE"], "write_kb_per_dispatch": per[k]["WRITE_SIZE"],
                        "copy_calibration": {"fetch_factor": ff, "write_factor": fw},
                        "rdreq_by_size": {c: per[k].get(c) for c in ["TCC_EA0_RDREQ_sum"] +
                                          [c for c, _ in RDREQ_SIZES]},
                        "rdreq_read_bytes_per_launch": rd,
                        "rdreq_over_fetch_scaled": rd / read_b if rd else None,
                        "copy_rdreq_bytes": copy_rd[0] if copy_rd else None,
                        "hbm_read_bytes_per_launch": read_b, "hbm_write_bytes_per_launch": write_b,
                        "hbm_bytes_per_launch": read_b + write_b, "commands": cmds}
                try:
                    import synthetic as S

                    A, _ = S.config_c2()
                    W = m[0] * m[1]
                    NP = -(-A.n // (kPanelBytes // 4))
                    data["long_min"] = max(W, 16 * NP)
                    data["nnz"] = A.nnz
                except Exception:  # noqa: BLE001
                    pass
                with open(TRAFFIC_FILE, "w") as f:
                    json.dump(data, f, indent=1)
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
    ap.add_argument("--schedule", default="planned",
                    help="headline schedule: planned (default: lb_spmv_planned, short rows on the merge path and "
                         "long rows on LDS panels of x), merge_path, auto (autotuned), group_mapped, thread_mapped")
    ap.add_argument("--long-min", type=int, default=0, help="planned: long-row threshold (0 = the plan's default)")
    ap.add_argument("--panel-blocks", type=int, default=0, help="planned: blocks per panel (0 = default)")
    ap.add_argument("--streams", type=int, default=0, help="planned: 1 or 2 streams (0 = default, 1)")
    ap.add_argument("--graph", action="store_true",
                    help="time the headline's K steps as one HIP graph replay instead of eager launches")
    ap.add_argument("--pmc-calib", action="store_true",
                    help="also run one 256 MiB device copy (known bytes) to scale rocprofv3 FETCH/WRITE_SIZE")
    ap.add_argument("--only", default="",
                    help="comma-separated sections to run without the headline: " + ", ".join(sorted(SECTIONS)))
    ap.add_argument("--graph-only", action="store_true",
                    help="run only the graph traversals (SSSP, BFS) and print their figures")
    ap.add_argument("--record", metavar="FILE",
                    help="append one JSONL record per finished section (and the headline) to FILE")
    ap.add_argument("--resume", action="store_true",
                    help="with --record: read back sections FILE holds for the same kernel sources and device "
                         "instead of measuring them again")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="write profiles/ summaries from rocprofv3 CSV output under DIR and exit")
    args = ap.parse_args()
    if args.resume and not args.record:
        print("--resume needs --record FILE", file=sys.stderr)
        return 2
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
    props = torch.cuda.get_device_properties(dev)
    rec = Records(args.record, args.resume, f"{props.gcnArchName} {props.multi_processor_count} CUs")
    if args.graph_only:
        print(json.dumps({"graph_powerlaw1M": run_graph(lb, S, dev, args.no_cpu)}), flush=True)
        return 0
    stream = torch.cuda.current_stream(dev)
    flush = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB, larger than L2 + MALL
    sink = torch.empty((), dtype=torch.float32, device=dev)

    def evict():
        """Evict L2 and the Infinity Cache by reading the 1 GiB buffer (cached
        loads): the lines left behind are clean, so the next call pays for its
        own misses only, not for another buffer's write-back."""
        torch.sum(flush, dim=0, out=sink)

    if args.pmc_calib:  # a device copy of known size for the counter runs' calibration
        src = torch.ones(1 << 26, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        lb.probe_copy(src, dst)  # reads and writes exactly 256 MiB, as probe_copy_kernel
        torch.cuda.synchronize()
        del src, dst

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

    def cold(fn, reps, write=False):
        """median ms of single calls, each after a 1 GiB read (or, with write,
        a 1 GiB write) that evicts L2 and MALL."""
        out = []
        for r in range(reps):
            if write:
                flush.fill_(1.0)
            else:
                evict()
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

    result = {}
    value = None
    if args.only:
        wanted = set(args.only.split(","))
        unknown = wanted - SECTIONS
        if unknown:
            print(f"unknown sections {sorted(unknown)}; choose from {sorted(SECTIONS)}", file=sys.stderr)
            return 2
        if wanted & {"schedules", "bf16"}:  # the headline matrix, untimed
            A, x = S.config_c2()
            Ad = lb.CSR.from_host(A, dev)
            xd = torch.from_numpy(x).to(dev)
            y = torch.empty(A.m, dtype=torch.float32, device=dev)
            B = spmv_bytes(A.m, A.n, A.nnz)
    else:
        wanted = None
        # ------------------------------------------------------------ headline workload
        t0 = time.time()
        A, x = S.config_c2()
        log(f"[bench] power-law 2M generated: nnz={A.nnz} in {time.time() - t0:.1f}s")
        Ad = lb.CSR.from_host(A, dev)
        xd = torch.from_numpy(x).to(dev)
        y = torch.empty(A.m, dtype=torch.float32, device=dev)
        B = spmv_bytes(A.m, A.n, A.nnz)
        params = {}
        if args.items:
            params["items_per_thread"] = args.items
        if args.block:
            params["block_size"] = args.block
        head = args.schedule
        plan_info, plan_build_ms = None, None
        if head == "planned":
            if args.x_bands:
                params["x_bands"] = args.x_bands
            for k, v in (("long_min", args.long_min), ("panel_blocks", args.panel_blocks), ("streams", args.streams)):
                if v:
                    params[k] = v
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan = lb.Plan(Ad, **params)  # once per pattern: reads row_offsets through the host
            torch.cuda.synchronize()
            plan_build_ms = (time.perf_counter() - t0) * 1e3
            plan_info = plan.info
            ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device=dev)
            log(f"[bench] plan built in {plan_build_ms:.1f} ms: {plan_info}")

            def step():
                lb.spmv_planned(Ad, plan, xd, y=y, workspace=ws)
            sched = {"schedule": "planned", **{k: plan_info[k] for k in
                     ("block_size", "items_per_thread", "x_bands", "long_min", "panel_cols", "panel_blocks", "streams")}}
            kernels = ["merge_consume", "panel_consume", "plan_finish"]
        else:
            if args.x_bands and head == "merge_path":
                params["x_bands"] = args.x_bands
            if head == "auto" and not params:
                lb.autotune_clear()
                t0 = time.time()
                lb.tune(Ad)  # schedule and tile size picked by timing the candidates on this matrix
                log(f"[bench] autotuned in {time.time() - t0:.1f}s")
            elif head == "auto":
                head = "merge_path"
            sched = lb.resolve_schedule(Ad, head, **params)
            ws = torch.empty(max(lb.workspace_size(Ad, head, **params), 1), dtype=torch.uint8, device=dev)

            def step():
                lb.spmv(Ad, xd, head, y=y, workspace=ws, **params)
            kernels = {"merge_path": ["merge_consume", "merge_partition",
                                      "merge_finish" if sched["x_bands"] == 2 else "merge_fixup"],
                       "group_mapped": ["group_mapped"], "thread_mapped": ["thread_mapped"]}[sched["schedule"]]

        # bring the GPU's clocks up before the W warm-up steps: about 0.3 s of
        # untimed steps (a cold GPU times the first hundred calls a few % slow)
        t_end = time.time() + 0.3
        while time.time() < t_end:
            for _ in range(20):
                step()
            torch.cuda.synchronize()
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        # The K timed steps: each reads 1 GiB first (evicting L2 and the Infinity
        # Cache, outside its events), then one call between events on the launch
        # stream.  ms_per_step is their median: the cold figure.
        per_step = []
        t_region = time.perf_counter()
        for r in range(args.steps):
            evict()
            a_ev = torch.cuda.Event(enable_timing=True)
            b_ev = torch.cuda.Event(enable_timing=True)
            a_ev.record(stream)
            step()
            b_ev.record(stream)
            torch.cuda.synchronize()
            per_step.append(a_ev.elapsed_time(b_ev))
        region_s = time.perf_counter() - t_region
        ms = float(np.median(per_step))
        timing = "cold median"
        ms_cold_write = cold(step, args.steps, write=True)  # the same after a 1 GiB write
        ms_warm = timed(step, args.steps, 2)  # back to back, caches warm
        ms_graph = None
        if args.graph:
            ms_graph = graph_timed(step, y, args.steps)
        value = B / (ms * 1e-3) / 1e9
        log(f"[bench] {sched}: cold {ms * 1e3:.1f} us/step (median of {args.steps}), warm {ms_warm * 1e3:.1f} us, "
            f"{value:.0f} GB/s")
        kt = {n: kernel_avg_ms(step, args.steps, n) for n in kernels}
        kt = {n: v for n, v in kt.items() if v[1] > 0}
        dominant = max(kt, key=lambda n: kt[n][0])
        dom_ms, launches = kt[dominant]
        # algorithmic bytes of each kernel of the call (the planned call's parts)
        lens = np.diff(A.row_offsets.astype(np.int64))
        kernel_bytes = {}
        if head == "planned":
            long_nnz = int(plan_info["long_nnz"])
            short_nnz = A.nnz - long_nnz
            kernel_bytes["merge_consume"] = short_nnz * 8 + (A.m + 1) * 4 + A.m * 4 + A.n * 4
            kernel_bytes["panel_consume"] = long_nnz * 8 + A.n * 4 + int(plan_info["tasks"]) * 4
            kernel_bytes["plan_finish"] = (int(plan_info["tasks"]) * 4 + int(plan_info["long_rows"]) * 4 +
                                           (A.m * 12 + A.m // 8 if int(plan_info["x_bands"]) == 2 else 0))
        else:
            kernel_bytes[dominant] = B
        B_dom = kernel_bytes.get(dominant, B)
        achieved = B_dom / (dom_ms * 1e-3) / 1e9

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
        short_gather_ms = None
        if head == "planned":
            short_mask = np.repeat(lens < int(plan_info["long_min"]), lens)
            sidx = torch.from_numpy(np.ascontiguousarray(A.col_idx[short_mask])).to(dev)
            short_gather_ms, _ = kernel_avg_ms(
                lambda: lb.probe_gather(sidx, xd, pout, bands=plan_info["x_bands"]), 5, "probe_gather")
            ceilings["short_rows_gather_only_ms"] = round(short_gather_ms, 5)
            ceilings["short_rows_note"] = ("the same gather over the short rows' columns only, in the planned "
                                           "short-row consume's band form: the floor of that kernel")
            del sidx
        log(f"[bench] ceilings: {ceilings}")

        traffic, traffic_cfg = None, None
        if os.path.exists(TRAFFIC_FILE):
            try:
                with open(TRAFFIC_FILE) as f:
                    tr = json.load(f)
                same = (tr.get("schedule") == sched["schedule"] and tr.get("kernel") == dominant and
                        tr.get("kernel_source_hash") == kernel_source_hash() and tr.get("nnz") == A.nnz and
                        all(tr.get(k) == sched.get(k) for k in ("block_size", "items_per_thread", "x_bands", "long_min")))
                if same:
                    traffic = tr.get("hbm_bytes_per_launch")
                    traffic_cfg = {k: tr.get(k) for k in ("schedule", "block_size", "items_per_thread", "x_bands",
                                                         "long_min")}
                    traffic_cfg["unscaled_bytes"] = round((tr.get("fetch_kb_per_dispatch", 0) +
                                                           tr.get("write_kb_per_dispatch", 0)) * 1024)
                    # the read bytes counted by request size, over the copy-scaled FETCH_SIZE
                    traffic_cfg["rdreq_over_fetch_scaled"] = tr.get("rdreq_over_fetch_scaled")
            except (OSError, ValueError):
                traffic = None

        ceiling_key = "gather_bound_2band_gbs" if sched.get("x_bands") == 2 else "gather_bound_gbs"
        roofline = {"kernel": dominant, "bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / PEAK_GBS, 4), "traffic": traffic, "traffic_profiled_config": traffic_cfg,
                    "avg_launch_ms": round(dom_ms, 5), "launches": launches,
                    "algorithmic_bytes_per_launch": B_dom,
                    "kernels_ms": {n: round(v[0], 5) for n, v in kt.items()},
                    "kernels_gbs": {n: round(kernel_bytes[n] / (kt[n][0] * 1e-3) / 1e9, 1)
                                    for n in kt if n in kernel_bytes}}
        # the whole call on the same footing: B over the cold and warm step times
        roofline["call"] = {"bytes": B, "cold_gbs": round(B / (ms * 1e-3) / 1e9, 1),
                            "cold_frac": round(B / (ms * 1e-3) / 1e9 / PEAK_GBS, 4),
                            "warm_gbs": round(B / (ms_warm * 1e-3) / 1e9, 1),
                            "warm_frac": round(B / (ms_warm * 1e-3) / 1e9 / PEAK_GBS, 4)}
        if head == "planned" and short_gather_ms:
            roofline["gather_floor_ms"] = round(short_gather_ms, 5)
            roofline["frac_of_gather_floor"] = round(short_gather_ms / dom_ms, 4) if dominant == "merge_consume" else None
            roofline["note"] = ("the dominant kernel is the short rows' consume: about 9 nonzeros per row with "
                                "uniformly random columns, one random x gather per nonzero, so the gather request "
                                "rate, not HBM, bounds it (gather_floor_ms: the gather alone over the same columns in "
                                "the same band form); the long rows' panel kernel streams at "
                                "kernels_gbs.panel_consume; call: the whole call against 8 TB/s")
        else:
            roofline["gather_ceiling_gbs"] = ceilings[ceiling_key]
            roofline["frac_of_gather_ceiling"] = round(achieved / ceilings[ceiling_key], 4)

        cfg = {"workload": "powerlaw_m2M_zipf1.8_cap200k_empty10pct", "m": A.m, "n": A.n, "nnz": A.nnz, "seed": 2,
               **sched}
        result = {
            "metric": METRIC,
            "value": round(value, 2),
            "unit": "GB/s",
            "n_gpus": 1,
            "steps": args.steps,
            "warmup": args.warmup,
            "ms_per_step": round(ms, 5),
            "timing": timing,
            "cold_write_flush_ms": round(ms_cold_write, 5),
            "warm_ms_per_step": round(ms_warm, 5),
            "warm_gbs": round(B / (ms_warm * 1e-3) / 1e9, 2),
            "timed_region_s": round(region_s, 3),
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f32",
            "data": "synthetic",
            "config": cfg,
            "pct_of_peak": round(100 * value / PEAK_GBS, 2),
            "gflops": round(2 * A.nnz / (ms * 1e-3) / 1e9, 2),
            "algorithmic_bytes": B,
            "ceilings": ceilings,
            "roofline": roofline,
            "host": host_facts(),
        }
        if ms_graph is not None:
            result["hip_graph_ms_per_step"] = round(ms_graph, 5)
        if plan_info is not None:
            result["plan"] = {"build_ms": round(plan_build_ms, 2), "plan_bytes": int(plan_info["plan_bytes"]),
                              "workspace_bytes": int(plan_info["workspace_bytes"]),
                              **{k: int(plan_info[k]) for k in ("long_rows", "long_nnz", "panels", "tasks", "units",
                                                                  "active_units")},
                              "note": "built once per sparsity pattern, outside the timed region; values and x may "
                                      "change between calls"}
            # the same matrix on the unplanned merge path (two column bands), cold and warm
            wsu = torch.empty(max(lb.workspace_size(Ad, "merge_path", x_bands=2), 1), dtype=torch.uint8, device=dev)
            fu = (lambda: lb.spmv(Ad, xd, "merge_path", y=y, workspace=wsu, x_bands=2))
            tu = timed(fu, args.steps, 2)
            tuc = cold(fu, 10)
            result["merge_path_unplanned"] = {"warm_ms": round(tu, 5), "cold_ms": round(tuc, 5),
                                              "cold_gbs": round(B / (tuc * 1e-3) / 1e9, 2),
                                              "warm_gbs": round(B / (tu * 1e-3) / 1e9, 2)}
            del wsu

        # ------------------------------------------------------------ CPU oracle baseline
        if not args.no_cpu:
            import oracle

            orc = oracle.default()
            y_ref = orc.spmv(A.row_offsets, A.col_idx, A.values, x)  # warm-up (its result checks the GPU's below)
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
            # accuracy of the headline's output (outside the timed region) against the oracle's
            scale = orc.spmv(A.row_offsets, A.col_idx, A.values, x, abs_terms=True)
            step()
            torch.cuda.synchronize()
            err = np.abs(y.cpu().numpy().astype(np.float64) - y_ref)
            ratio = float(np.max(err / np.where(scale > 0, scale, 1.0)))
            result["accuracy"] = {"max_err_over_sum_abs_terms": ratio, "tolerance": 1e-5,
                                  "zero_rows_exact": bool(np.all(err[scale == 0] == 0))}
            log(f"[bench] cpu oracle: {cpu_s * 1e3:.0f} ms/call on {orc.num_threads()} threads; max err ratio {ratio:.2e}")
        rec.append("headline", dict(result))
        if args.quick:
            print(json.dumps(result), flush=True)
            return 0

    resumed = []

    def want(name):
        if wanted is not None and name not in wanted:
            return False
        if name in rec.done:  # measured by an earlier run of the same kernels on this device
            result[SECTION_KEYS[name]] = rec.done[name]
            resumed.append(name)
            return False
        return True

    def finish(name):
        rec.append(name, result[SECTION_KEYS[name]])


    extra_steps = max(3, min(args.steps, 10))

    if want("schedules"):
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
        finish("schedules")

    if want("uniform"):
        # ------------------------------------------------------------ the small uniform matrix (launch-bound)
        A1, x1 = S.config_c1()
        A1d = lb.CSR.from_host(A1, dev)
        x1d = torch.from_numpy(x1).to(dev)
        y1 = torch.empty(A1.m, dtype=torch.float32, device=dev)
        small = {"m": A1.m, "nnz": A1.nnz,
                 "note": "us per call: eager back-to-back calls from Python (bound by the host's per-call work), "
                         "and hip_graph_us: 100 calls captured in one HIP graph and replayed (the GPU's own time "
                         "per call, launch gaps included); accuracy is asserted by the GPU tests",
                 "hip_graph_us": {}}
        calls = []
        for name, p in (("thread_mapped", {}), ("group_mapped", {"group_size": 64}),
                        ("group_mapped", {"group_size": 64, "tiles_per_group": 64}), ("merge_path", {})):
            ws1 = torch.empty(max(lb.workspace_size(A1d, name, **p), 1), dtype=torch.uint8, device=dev)
            key = name + ("" if not p else "_" + "_".join(f"{k}{v}" for k, v in p.items()))
            calls.append((key, lambda name=name, p=p, ws1=ws1: lb.spmv(A1d, x1d, name, y=y1, workspace=ws1, **p)))
        small["merge_path_units"] = {k: v for k, v in lb.resolve_schedule(A1d, "merge_path").items()
                                     if k in ("block_size", "items_per_thread")}
        pl1 = lb.Plan(A1d)
        wsp1 = torch.empty(max(pl1.workspace_bytes, 1), dtype=torch.uint8, device=dev)
        calls.append(("planned", lambda: lb.spmv_planned(A1d, pl1, x1d, y=y1, workspace=wsp1)))
        for key, f in calls:
            small[key] = round(timed(f, 50, 10) * 1e3, 2)
            tg = graph_timed(f, y1, 100)
            small["hip_graph_us"][key] = round(tg * 1e3, 2) if tg is not None else None
        result["uniform4096"] = small
        finish("uniform")
        log(f"[bench] uniform 4096: {small}")
        del A1d, x1d, y1

    if want("bf16"):
        # ------------------------------------------------------------ BF16 (accuracy is asserted by the GPU tests)
        bf = {}
        Ab = A.with_values(S.to_bf16_bits(A.values))
        xb = S.to_bf16_bits(x)
        Abd = lb.CSR.from_host(Ab, dev)
        xbd = torch.from_numpy(xb.view(np.int16).copy()).view(torch.bfloat16).to(dev)
        wsb = torch.empty(lb.workspace_size(Abd, "merge_path"), dtype=torch.uint8, device=dev)
        t = timed(lambda: lb.spmv(Abd, xbd, "merge_path", y=y, workspace=wsb), extra_steps, 2)
        Bb = spmv_bytes(A.m, A.n, A.nnz, 2, 2)
        bf["powerlaw2M"] = {"ms": round(t, 4), "gbs": round(Bb / (t * 1e-3) / 1e9, 2),
                            "fp32_gbs": round(value, 2) if value else None}
        plb = lb.Plan(Abd)  # the planned call in BF16 (panels of 81920 BF16 columns)
        wspb = torch.empty(max(plb.workspace_bytes, 1), dtype=torch.uint8, device=dev)
        fpb = (lambda: lb.spmv_planned(Abd, plb, xbd, y=y, workspace=wspb))
        tp, tpc = timed(fpb, extra_steps, 2), cold(fpb, 10)
        bf["powerlaw2M"]["planned"] = {"warm_ms": round(tp, 4), "warm_gbs": round(Bb / (tp * 1e-3) / 1e9, 2),
                                       "cold_ms": round(tpc, 4), "cold_gbs": round(Bb / (tpc * 1e-3) / 1e9, 2),
                                       "long_rows": plb.info["long_rows"], "long_nnz": plb.info["long_nnz"]}
        del Abd, xbd, plb, wspb
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
        # planned: no long rows here, so the merge path with the split precomputed (one launch fewer)
        for key, Md, xmd, Bm in (("fp32", Ld, xld, BL), ("bf16", Lbd, xlbd, BLb)):
            plm = lb.Plan(Md)
            wsp = torch.empty(max(plm.workspace_bytes, 1), dtype=torch.uint8, device=dev)
            fp = (lambda Md=Md, xmd=xmd, plm=plm, wsp=wsp: lb.spmv_planned(Md, plm, xmd, y=yl, workspace=wsp))
            tp, tpc = timed(fp, extra_steps, 2), cold(fp, 10)
            bf["laplacian2048"][f"{key}_planned"] = {"warm_ms": round(tp, 4), "warm_gbs": round(Bm / (tp * 1e-3) / 1e9, 2),
                                                     "cold_ms": round(tpc, 4),
                                                     "cold_gbs": round(Bm / (tpc * 1e-3) / 1e9, 2),
                                                     "long_rows": plm.info["long_rows"]}
            del plm, wsp
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
        finish("bf16")
        log(f"[bench] bf16: {bf}")
        del Ld, Lbd, xld, xlbd, yl

    if want("fwdbwd"):
        # ------------------------------------------------------------ forward + backward (1M)
        C4, x4 = S.config_c4()
        C4d = lb.CSR.from_host(C4, dev)
        x4d = torch.from_numpy(x4).to(dev)
        dy4 = torch.from_numpy(S.random_vector(44, C4.m)).to(dev)
        y4 = torch.empty(C4.m, dtype=torch.float32, device=dev)
        ws4 = torch.empty(lb.workspace_size(C4d, "merge_path"), dtype=torch.uint8, device=dev)
        tf = timed(lambda: lb.spmv(C4d, x4d, "merge_path", y=y4, workspace=ws4), extra_steps, 2)
        pl4 = lb.Plan(C4d)
        wsp4 = torch.empty(max(pl4.workspace_bytes, 1), dtype=torch.uint8, device=dev)
        tfp = timed(lambda: lb.spmv_planned(C4d, pl4, x4d, y=y4, workspace=wsp4), extra_steps, 2)
        del pl4, wsp4
        tb = timed(lambda: lb.spmv_backward(C4d, x4d, dy4), extra_steps, 2)
        bw_ms, _ = kernel_avg_ms(lambda: lb.spmv_backward(C4d, x4d, dy4), extra_steps, "backward")
        tr4 = lb.transpose_pattern(C4d.pattern)  # once per pattern; then its rebuild timed on the stream
        tbuild = timed(lambda: lb.transpose_pattern(C4d.pattern, rebuild=True), 5, 1)
        tr4 = lb.transpose_pattern(C4d.pattern)
        tbt = timed(lambda: lb.spmv_backward(C4d, x4d, dy4, transposed=tr4), extra_steps, 2)
        Bf4, Bb4 = spmv_bytes(C4.m, C4.n, C4.nnz), backward_bytes(C4.m, C4.n, C4.nnz)
        result["fwd_bwd_powerlaw1M"] = {"nnz": C4.nnz, "fwd_ms": round(tf, 4), "bwd_ms": round(tb, 4),
                                        "fwd_planned_ms": round(tfp, 4),
                                        "fwd_planned_gbs": round(spmv_bytes(C4.m, C4.n, C4.nnz) / (tfp * 1e-3) / 1e9, 2),
                                        "fwd_gbs": round(Bf4 / (tf * 1e-3) / 1e9, 2),
                                        "bwd_gbs": round(Bb4 / (tb * 1e-3) / 1e9, 2),
                                        "bwd_kernel_ms": round(bw_ms, 4),
                                        "bwd_transposed_ms": round(tbt, 4),
                                        "bwd_transposed_gbs": round(Bb4 / (tbt * 1e-3) / 1e9, 2),
                                        "transpose_build_ms": round(tbuild, 3),
                                        "fwd_bwd_transposed_gbs": round((Bf4 + Bb4) / ((tf + tbt) * 1e-3) / 1e9, 2),
                                        "fwd_bwd_gbs": round((Bf4 + Bb4) / ((tf + tb) * 1e-3) / 1e9, 2)}
        finish("fwdbwd")
        log(f"[bench] fwd+bwd: {result['fwd_bwd_powerlaw1M']}")

    if want("formats"):
        # ------------------------------------------------------------ other tile sets (1M): COO and CSC
        if "C4d" not in locals():  # the 1M matrix and its CSR forward, when fwdbwd did not run
            C4, x4 = S.config_c4()
            C4d = lb.CSR.from_host(C4, dev)
            x4d = torch.from_numpy(x4).to(dev)
            y4 = torch.empty(C4.m, dtype=torch.float32, device=dev)
            ws4 = torch.empty(lb.workspace_size(C4d, "merge_path"), dtype=torch.uint8, device=dev)
            dy4 = None
            tf = timed(lambda: lb.spmv(C4d, x4d, "merge_path", y=y4, workspace=ws4), extra_steps, 2)
            Bf4 = spmv_bytes(C4.m, C4.n, C4.nnz)
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
        finish("formats")
        log(f"[bench] formats: {fm}")
        del C4d, x4d, dy4, y4, ws4

    if want("batched"):
        # ------------------------------------------------------------ batched (512 matrices)
        t0 = time.time()
        BH = S.config_c5()
        log(f"[bench] batched generated: {BH.count} matrices, nnz={BH.nnz} in {time.time() - t0:.1f}s")
        Bd = lb.Batch.from_host(BH, dev)
        bres = {"count": BH.count, "total_rows": BH.total_rows, "nnz": BH.nnz}
        # context: the same products as one lb_spmm call per matrix (merge
        # path, default tiles) on views of the batch's arrays
        rb, zb, cb = (t.cpu().tolist() for t in (Bd.mat_row_base, Bd.mat_nnz_base, Bd.mat_col_base))
        mats = [lb.CSR(Bd.row_offsets[rb[b]:rb[b + 1] + 1] - zb[b], Bd.col_idx[zb[b]:zb[b + 1]],
                       Bd.values[zb[b]:zb[b + 1]], (rb[b + 1] - rb[b], cb[b + 1] - cb[b])) for b in range(BH.count)]
        wsl = torch.empty(max(lb.workspace_size(M, "merge_path", k=kk) for M in mats for kk in (1, 8)),
                          dtype=torch.uint8, device=dev)
        for k in (1, 8):
            Xk = torch.from_numpy(S.random_vector(55, BH.total_cols * k).reshape(-1, k)).to(dev)
            Yk = torch.empty((BH.total_rows, k), dtype=torch.float32, device=dev)
            tuned = lb.tune_batched(Bd, k)
            tk = timed(lambda: lb.batched_spmm(Bd, Xk, "auto", Y=Yk), extra_steps, 2)
            Bk = BH.nnz * 8 + (BH.total_rows + 1) * 4 + BH.total_cols * 4 * k + BH.total_rows * 4 * k
            bres[f"k{k}"] = {"ms": round(tk, 4), "gbs": round(Bk / (tk * 1e-3) / 1e9, 2),
                             "gflops": round(2 * BH.nnz * k / (tk * 1e-3) / 1e9, 2), "schedule": tuned}

            def per_matrix(Xk=Xk, Yk=Yk):
                for b, M in enumerate(mats):
                    lb.spmm(M, Xk[cb[b]:cb[b + 1]], "merge_path", Y=Yk[rb[b]:rb[b + 1]], workspace=wsl)

            tl = timed(per_matrix, 3, 1)
            tlg = graph_timed(per_matrix, Yk, 1)
            bres[f"k{k}"]["per_matrix_loop"] = {
                "ms": round(tl, 4), "gbs": round(Bk / (tl * 1e-3) / 1e9, 2),
                "hip_graph_ms": round(tlg, 4) if tlg is not None else None,
                "note": f"{BH.count} lb_spmm calls, one per matrix (merge path), eager from Python and as one "
                        "HIP graph replay"}
            del Xk, Yk
            log(f"[bench] batched k={k}: {bres[f'k{k}']}")
        del mats, wsl
        result["batched_512"] = bres
        finish("batched")
        del Bd

    if want("graph"):
        result["graph_powerlaw1M"] = run_graph(lb, S, dev, args.no_cpu)
        finish("graph")

    if want("spgemm"):
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
        finish("spgemm")
        log(f"[bench] spgemm: {gm}")

    if resumed:
        result["resumed_sections"] = resumed
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
