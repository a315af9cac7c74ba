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
