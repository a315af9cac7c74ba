"""include/lb.h compiles as C11 and liblb.so links and answers host-only
calls from a plain C program (no GPU needed)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2301_04792_amd")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_c_program_uses_the_abi(tmp_path):
    if not os.path.exists(os.path.join(LIBDIR, "liblb.so")):
        pytest.skip("liblb.so not built")
    exe = tmp_path / "c_abi_check"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c_abi_check.c"), "-L", LIBDIR, "-llb",
                    f"-Wl,-rpath,{LIBDIR}", "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "ok"


def test_bench_refuses_several_gpus():
    r = subprocess.run(["python", os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_bench_records_resume(tmp_path):
    """bench.py's JSONL records: each finished section is appended with the
    kernel sources' hash and the device; with resume, only sections recorded
    for the same sources and device are read back, and a line cut short by an
    interrupted run is skipped."""
    import importlib.util

    spec = importlib.util.spec_from_file_location("_bench", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    path = tmp_path / "records.jsonl"
    w = bench.Records(str(path), False, "gfx950 256 CUs")
    w.append("headline", {"value": 1.0})
    w.append("uniform", {"planned": 7.8})
    w.append("batched", {"k1": {"ms": 1.1}})
    bench.Records(str(path), False, "gfx942 304 CUs").append("schedules", {"merge_path": {"ms": 0.4}})
    with open(path, "a") as f:
        f.write('{"section": "spgemm", "kernel_sources": "')  # the run stopped mid-line
    r = bench.Records(str(path), True, "gfx950 256 CUs")
    assert r.done == {"uniform": {"planned": 7.8}, "batched": {"k1": {"ms": 1.1}}}  # no headline, no other device
    assert bench.Records(str(path), False, "gfx950 256 CUs").done == {}  # resume off: nothing read back
    lines = path.read_text().splitlines()
    assert len(lines) == 5
    import json

    first = json.loads(lines[0])
    assert first["section"] == "headline" and first["kernel_sources"] == bench.kernel_source_hash()
    assert set(first["host"]) == {"cpu_model", "logical_cpus"}


def test_bench_resume_needs_record():
    r = subprocess.run(["python", os.path.join(ROOT, "bench.py"), "--resume"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "--record" in r.stderr


def test_profile_summary_counts_reads_by_request_size(tmp_path, monkeypatch):
    """The counter summary turns the per-size L2 read requests into bytes
    (32, 64 and 128 per request, no scale factor) and checks them on the
    calibration copy; the headline's traffic record keeps FETCH_SIZE and
    WRITE_SIZE scaled by the copy and reports the size-counted reads beside
    them."""
    import csv
    import importlib.util
    import json

    import synthetic

    spec = importlib.util.spec_from_file_location("_bench", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    traffic = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(traffic))
    monkeypatch.setattr(synthetic, "config_c2", lambda: (synthetic.config_c1()[0], None))
    consume = "void lbk::merge_spmv_consume<128, 8, float, float, 2, false, 1, true>(int, int)"
    copy = "lbk::probe_copy_kernel(float const*, float*, long)"
    # the copy reads 2^28 bytes in 128-byte requests: FETCH_SIZE sees half
    copy_vals = {"FETCH_SIZE": 131072.0, "WRITE_SIZE": 262144.0, "TCC_EA0_RDREQ_sum": 2.0 ** 21,
                 "TCC_EA0_RDREQ_32B_sum": 0.0, "TCC_EA0_RDREQ_64B_sum": 0.0, "TCC_EA0_RDREQ_128B_sum": 2.0 ** 21}
    cons_vals = {"FETCH_SIZE": 300000.0, "WRITE_SIZE": 20000.0, "TCC_EA0_RDREQ_sum": 5.0e6,
                 "TCC_EA0_RDREQ_32B_sum": 1.0e6, "TCC_EA0_RDREQ_64B_sum": 3.0e6, "TCC_EA0_RDREQ_128B_sum": 0.9e6}
    tag = "planned_spmv_powerlaw2M"
    for i, cset in enumerate(bench.COUNTERS[tag][1]):
        names = cset.split()
        d = tmp_path / "prof" / f"{tag}_{i}" / "host"
        d.mkdir(parents=True)
        with open(d / "c_counter_collection.csv", "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
            w.writeheader()
            for kname, vals in ((copy, copy_vals), (consume, cons_vals)):
                for c in names:
                    for _ in range(3 if kname == consume else 1):
                        w.writerow({"Kernel_Name": kname, "Counter_Name": c, "Counter_Value": vals.get(c, 1.0)})
    bench.summarize_profiles(str(tmp_path / "profiles"), str(tmp_path / "prof"))
    md = (tmp_path / "profiles" / f"{tag}_counters.md").read_text()
    assert "On the calibration copy they give 2.68435e+08 bytes against the 2^28 = 2.68435e+08" in md
    assert "rdreq_bytes" in md and "rdreq_unsized" in md
    t = json.loads(traffic.read_text())
    want_read = 32 * 1.0e6 + 64 * 3.0e6 + 128 * 0.9e6
    fetch = 300000.0 * 1024 * 2.0  # the copy's FETCH_SIZE is half its bytes: factor 2
    assert t["hbm_read_bytes_per_launch"] == fetch
    assert t["rdreq_read_bytes_per_launch"] == want_read
    assert abs(t["rdreq_over_fetch_scaled"] - want_read / fetch) < 1e-12
    assert t["hbm_write_bytes_per_launch"] == 20000.0 * 1024
    assert t["hbm_bytes_per_launch"] == fetch + 20000.0 * 1024
    assert t["copy_rdreq_bytes"] == 2.0 ** 28
    assert t["kernel_source_hash"] == bench.kernel_source_hash()
