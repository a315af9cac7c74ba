"""The tuning cache on the device: pattern fingerprints, per-pattern picks,
bindings for schedule="auto", and the cache file across processes."""
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

import synthetic as S
import synthetic.csr as SC

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2301_04792_amd as lb  # noqa: E402

DEV = "cuda:0"
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_fingerprint_follows_the_pattern_only():
    A, _ = S.powerlaw_csr(71, 50_000, 50_000, 1.8, 5_000, 0.1)
    Ad = lb.CSR.from_host(A, DEV)
    f1 = lb.pattern_fingerprint(Ad)
    assert f1 == lb.pattern_fingerprint(Ad)
    # new values, same pattern: same fingerprint
    A2 = A.with_values(S.random_vector(72, A.nnz, role=3))
    assert lb.pattern_fingerprint(lb.CSR.from_host(A2, DEV)) == f1
    # same shape and nnz, the longest row's columns shifted by one: another pattern
    r = int(np.argmax(np.diff(A.row_offsets)))
    lo, hi = int(A.row_offsets[r]), int(A.row_offsets[r + 1])
    ci = A.col_idx.copy()
    ci[lo:hi] = np.minimum(A.col_idx[lo:hi] + 1, A.n - 1)
    B = SC.CSRHost(A.row_offsets, ci, A.values, A.shape)
    assert lb.pattern_fingerprint(lb.CSR.from_host(B, DEV)) != f1
    # same shape and nnz, different row lengths
    ro = A.row_offsets.copy()
    k = int(np.flatnonzero(np.diff(ro) > 1)[0])
    ro[k + 1] -= 1
    C = SC.CSRHost(ro, A.col_idx, A.values, A.shape)
    assert lb.pattern_fingerprint(lb.CSR.from_host(C, DEV)) != f1


def test_tuned_pick_binds_to_its_pattern():
    """A pick tuned for one pattern does not leak to another matrix of the
    same shape: that one gets the Sec. 6.2 rule until it is tuned or looked
    up itself."""
    A, x = S.powerlaw_csr(73, 60_000, 60_000, 1.8, 8_000, 0.1)
    Ad = lb.CSR.from_host(A, DEV)
    B = SC.CSRHost(A.row_offsets, np.ascontiguousarray(A.col_idx[::-1]), A.values, A.shape)  # same shape
    Bd = lb.CSR.from_host(B, DEV)
    fa, fb = lb.pattern_fingerprint(Ad), lb.pattern_fingerprint(Bd)
    assert fa != fb
    lb.autotune_clear()
    best = lb.tune(Ad)
    assert lb.resolve_schedule(Ad, "auto") == best
    rule = lb.resolve_schedule(Bd, "auto")  # unbound
    assert rule["schedule"] == "merge_path" and rule["items_per_thread"] == 8 and rule["block_size"] == 256
    assert rule["x_bands"] == 1 and rule["vector_width"] == 1
    assert lb.autotune_lookup(Bd, 1, fb) is None  # B's own pattern was never tuned
    assert lb.resolve_schedule(Bd, "auto") == rule
    # binding B to A's fingerprint (as a lookup would for A's pattern) gives A's pick
    assert lb.autotune_lookup(Bd, 1, fa) == best
    assert lb.resolve_schedule(Bd, "auto") == best
    lb.autotune_clear()
    assert lb.resolve_schedule(Ad, "auto") == rule


def test_cache_file_across_processes(tmp_path):
    """Process 1 tunes with LB_AUTOTUNE_CACHE set: the file gains an entry
    for this device and ABI and keeps a line of another ABI version.
    Process 2 finds the pick by fingerprint without tuning."""
    cache = tmp_path / "tune.txt"
    cache.write_text("lbtune 1 gfx000:1 10 10 10 1 0 0 1 2 0 0 8 256 0 1 1\n")
    prog = textwrap.dedent(f"""
        import sys, json
        sys.path.insert(0, {ROOT!r})
        import torch, synthetic as S
        import paper_2301_04792_amd as lb
        A, x = S.powerlaw_csr(74, 40_000, 40_000, 1.8, 4_000, 0.1)
        Ad = lb.CSR.from_host(A, "cuda:0")
        if sys.argv[1] == "tune":
            print(json.dumps(lb.tune(Ad)))
        else:
            print(json.dumps([lb.resolve_schedule(Ad, "auto"), lb.autotune_lookup(Ad, 1),
                              lb.resolve_schedule(Ad, "auto")]))
    """)
    env = dict(os.environ, LB_AUTOTUNE_CACHE=str(cache))
    r1 = subprocess.run([sys.executable, "-c", prog, "tune"], capture_output=True, text=True, env=env, timeout=300)
    assert r1.returncode == 0, r1.stderr[-2000:]
    lines = cache.read_text().splitlines()
    tag = lb._lib.lb_autotune_device_tag().decode()
    assert lines[0] == "lbtune 1 gfx000:1 10 10 10 1 0 0 1 2 0 0 8 256 0 1 1"
    assert any(l.startswith(f"lbtune {lb._abi.ABI_VERSION} {tag} 40000 40000 ") for l in lines[1:])
    r2 = subprocess.run([sys.executable, "-c", prog, "lookup"], capture_output=True, text=True, env=env, timeout=300)
    assert r2.returncode == 0, r2.stderr[-2000:]
    import json
    tuned = json.loads(r1.stdout.strip().splitlines()[-1])
    before, found, after = json.loads(r2.stdout.strip().splitlines()[-1])
    assert found == tuned and after == tuned
    assert before["items_per_thread"] == 8 and before["block_size"] == 256  # unbound: the Sec. 6.2 rule
